"""Benchmark of the DNN-MG fine-level correction step on one MI355X.

One step = prolongation -> fine residual -> patch gather -> patch network ->
multiplicity-averaged extension -> residual indicator (and, above its
threshold, the plain fine correction) -> right-hand side -> restriction (the
hot path after the coarse solve), captured in one HIP graph and replayed as a
time loop (each step's right-hand side feeds the next step's residual).

Headline workload: the large single run, channel 2.5 x 0.41 x 0.41 with
coarse 128x32x32 cells (131,072 patches) and fine 256x64x64 cells (1,085,825
nodes); FP32 stencils, network 165-512-512-81 with the E4M3 hidden product,
residual indicator with threshold 1 and the fallback to the plain fine
correction.  Its network is trained on the GPU (library kernels) on the plain
fine correction of four other seeded inputs of the same channel.  Prints one
JSON line; `value` is patches/s.  Also reported: the same step with FP32 and
BF16 networks, the 16,384-patch channel, the 32-box batch, a training step,
per-kernel rates, accuracy against the FP64 oracle and the oracle's own CPU
throughput.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3  # published vector FP32 (packed FMA); non-packed issue is half
BF16_MFMA_PEAK_TFLOPS = 2500.0
FP8_MFMA_PEAK_TFLOPS = 5000.0
PMC_COPY_MIB = 256  # plain copy of known size that calibrates the HBM byte counters
CPU_WORKERS = 16    # host threads / processes of the CPU baseline (the machine's CPU share per GPU)
DISTILL_SEEDS = (1, 2, 3, 4)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline and accuracy leg")
    ap.add_argument("--no-variants", action="store_true", help="only the headline workload")
    ap.add_argument("--profile-step", action="store_true",
                    help="run only the headline step's graph replays (for rocprofv3 --kernel-trace)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run only the headline step's dominant kernel and a plain copy (for rocprofv3 --pmc)")
    ap.add_argument("--scale-only", action="store_true",
                    help="run only the per-kernel measurements on the large channel (for rocprofv3)")
    ap.add_argument("--q2-step", action="store_true",
                    help="run only the Q2 step's graph replays on the large channel (for rocprofv3)")
    ap.add_argument("--profile-training", action="store_true",
                    help="run only the training-step variant for --steps steps (for rocprofv3)")
    ap.add_argument("--profile-paper-net", action="store_true",
                    help="run only the paper network form's step variant (for rocprofv3)")
    ap.add_argument("--profile-levels", action="store_true",
                    help="run only the two-level prediction's step variant (for rocprofv3)")
    ap.add_argument("--profile-batched", action="store_true",
                    help="run only the batched step of the 32 uneven boxes (for rocprofv3)")
    ap.add_argument("--cpu-worker", type=int, default=None, help=argparse.SUPPRESS)
    return ap.parse_args()


RESIDUAL_SOURCES = ("residual.hip", "common.hpp", "common.hip")
NETWORK_SOURCES = ("mlp.hip", "mlp.hpp", "lowp.hpp", "common.hpp", "common.hip")
# the sources each counted entry point is built from (a PMC summary holds
# for the sources it was taken on)
ENTRY_SOURCES = {"dnnmg_residual_b": RESIDUAL_SOURCES, "dnnmg_prolong_residual_b": RESIDUAL_SOURCES,
                 "dnnmg_residual_rhs_b": RESIDUAL_SOURCES,
                 "dnnmg_patch_gather_forward": NETWORK_SOURCES,
                 "dnnmg_q2_residual_b": ("q2.hip", "common.hpp", "common.hip")}


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
    if not k or k.get("src_hash") != src_hash(*ENTRY_SOURCES[entry]):
        return None
    return k.get("bytes_per_launch")


# ------------------------------------------------------------ CPU leg -------
def slab_workload():
    """The CPU sample: a slab of the large channel (its first 8 coarse cells
    along x, 8x32x32 coarse cells = 8,192 patches) at the same cell sizes,
    with the same network width."""
    import dnnmg_synth as syn

    w5 = syn.cfg5()
    box = syn.BoxSpec((8, 32, 32), (w5.box.len[0] * 8 / w5.box.n[0], w5.box.len[1], w5.box.len[2]), 0,
                      syn.CHANNEL_DIRICHLET)
    return syn.Workload("channel_slab_8x32x32_of_128x32x32", box, w5.ns, w5.hidden, "fp8", "channel")


def cpu_worker(seed):
    """One process of the CPU baseline: the oracle's full correction step with
    the indicator evaluated (the fallback not taken, as on the GPU), on the
    slab sample; prints its wall time."""
    import dnnmg_synth as syn
    import oracle

    w = slab_workload()
    inp = syn.step_inputs(w, seed=seed)
    params = [np.asarray(p, np.float32).astype(np.float64) for p in syn.mlp_params(165, w.hidden, 81, seed=seed)]
    oracle.lib()
    t0 = time.perf_counter()
    oracle.correction_step(w.box, w.ns, params, inp.xc, inp.vprev, indicator=True, theta=float("inf"))
    print(json.dumps({"seed": seed, "s": time.perf_counter() - t0}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def run_workers(n):
    t0 = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(k)],
                              stdout=subprocess.PIPE, text=True) for k in range(n)]
    outs = [p.communicate()[0] for p in procs]
    wall = time.perf_counter() - t0
    for p in procs:
        if p.returncode != 0:
            raise RuntimeError("CPU baseline worker failed")
    per = [json.loads(o.strip().splitlines()[-1])["s"] for o in outs]
    return wall, per


def cpu_baseline():
    """The oracle as it stands (single-threaded C), timed on the host before
    the GPU is touched: one process on the slab sample (one core), then
    CPU_WORKERS processes on CPU_WORKERS seeded slabs at once (all cores of
    the GPU's share)."""
    w = slab_workload()
    npch = w.box.n_patches
    wall1, _ = run_workers(1)
    wallN, per = run_workers(CPU_WORKERS)
    return {"value": npch / wall1, "unit": "patches/s", "cores": 1, "kind": "oracle",
            "sample": f"one full correction step (indicator evaluated, fallback not taken) of {w.name} "
                      f"({npch} patches, fine {2 * w.box.n[0]}x64x64 cells of the large channel, network width "
                      f"{w.hidden}) in FP64, {wall1:.1f} s on one core",
            "all_cores": {"value": CPU_WORKERS * npch / wallN, "unit": "patches/s", "cores": CPU_WORKERS,
                          "sample": f"{CPU_WORKERS} processes, each the same step on its own seeded slab, "
                                    f"{wallN:.1f} s wall (per process {min(per):.1f}-{max(per):.1f} s)"},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def oracle_reference(w, seed=0, threads=CPU_WORKERS):
    """FP64 oracle chain of one step (indicator evaluated, no fallback) on
    seeded inputs and seeded network weights: the reference of the accuracy
    figures (the network's rows on `threads` host threads)."""
    import dnnmg_synth as syn
    import oracle

    inp = syn.step_inputs(w, seed=seed)
    params = [np.asarray(p, np.float32).astype(np.float64) for p in syn.mlp_params(165, w.hidden, 81, seed=seed)]
    vp32 = np.asarray(inp.vprev, np.float32).astype(np.float64)
    t0 = time.perf_counter()
    ref = oracle.correction_step(w.box, w.ns, params, inp.xc, vp32, indicator=True, theta=float("inf"),
                                 threads=threads)
    keep = {k: ref[k] for k in ("xt", "r", "d", "bc", "eta")}
    keep["seconds"] = time.perf_counter() - t0
    return keep


# ------------------------------------------------------------ GPU leg -------
def time_graph(st, steps, warmup):
    """Graph replays of the step: `warmup` untimed, then `steps` timed with HIP
    events on the replay stream (one event between consecutive steps, for the
    median and minimum)."""
    import torch

    st.capture()
    for _ in range(warmup):
        st.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        st.replay()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    return {"ms": ev[0].elapsed_time(ev[steps]) / steps, "median_ms": float(np.median(per)),
            "min_ms": float(per.min()), "wall_s": wall}


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


def distilled_network(w):
    """The headline's network: trained on the GPU on the plain fine correction
    of DISTILL_SEEDS inputs of the same workload (train.distill)."""
    import dnnmg_synth as syn
    from paper_2307_14837_amd import train

    t0 = time.perf_counter()
    inputs = []
    for s in DISTILL_SEEDS:
        inp = syn.step_inputs(w, seed=s)
        inputs.append((inp.xc, inp.vprev))
    params, shift, inv, info = train.distill(w.box, w.ns, inputs, w.hidden, steps=600)
    info["seconds"] = time.perf_counter() - t0
    info["seeds"] = list(DISTILL_SEEDS)
    return params, shift, inv, info


def build_step(w, dtype, params=None, shift=None, inv=None, seed=0, indicator=False, theta=1.0):
    import dnnmg_synth as syn
    from paper_2307_14837_amd import stepper

    inp = syn.step_inputs(w, seed=seed)
    if params is None:
        params = syn.mlp_params(165, w.hidden, 81, seed=seed)
    st = stepper.CorrectionStep(w.box, w.ns, params, dtype=dtype, indicator=indicator, theta=theta,
                                shift=shift, inv_scale=inv)
    st.load(inp.xc, inp.vprev)
    return st, inp


def fallback_accounting(st, inp, steps):
    """The timed time loop replayed again from the same start, synchronising
    after each step to read the indicator: eta per step and how often the
    fallback was taken."""
    import torch

    st.load(inp.xc, inp.vprev)
    etas, taken = [], 0
    for _ in range(steps):
        st.replay()
        torch.cuda.synchronize()
        n = st.norms.cpu().numpy()
        etas.append(float(np.sqrt(n[1] / n[0])) if n[0] > 0 else 0.0)
        taken += int(st.fell_back.item())
    e = np.array(etas)
    return {"steps": steps, "fallback_rate": taken / steps, "eta_first": etas[0],
            "eta_median": float(np.median(e)), "eta_max": float(e.max())}


def run_step(w, dtype, steps, warmup, params=None, shift=None, inv=None, indicator=False, theta=1.0,
             account=False):
    st, inp = build_step(w, dtype, params, shift, inv, indicator=indicator, theta=theta)
    t = time_graph(st, steps, warmup)
    out = {"workload": w.name, "dtype": dtype, "indicator": indicator, "theta": theta if indicator else None,
           "ms_per_step": t["ms"], "median_ms": t["median_ms"], "min_ms": t["min_ms"],
           "patches_per_s": st.np / (t["ms"] * 1e-3), "fine_dof_per_s": 4 * st.nf / (t["ms"] * 1e-3)}
    if indicator and account:
        out["indicator_stats"] = fallback_accounting(st, inp, steps)
    return out, st, t


def run_levels(dtype, steps, warmup):
    """The two-level prediction on the large channel's fine mesh: coarse
    64x16x16 cells (16,384 patches of 4x4x4 fine cells), fine 256x64x64,
    network 753-512-512-375, indicator evaluated (threshold infinite: no
    fallback), seeded weights."""
    import dnnmg_synth as syn
    from paper_2307_14837_amd import stepper

    w5 = syn.cfg5()
    wc = syn.Workload("channel_64x16x16_two_levels", syn.channel_box((64, 16, 16)), w5.ns, 512, dtype, "channel")
    xc = syn.step_inputs(wc, seed=0).xc
    vprev = syn.step_inputs(w5, seed=0).vprev  # on the 256x64x64 fine lattice
    params = syn.mlp_params(753, 512, 375, seed=0)
    params[4] = params[4] * 0.05
    st = stepper.CorrectionStep(wc.box, wc.ns, params, dtype=dtype, levels=2, indicator=True, theta=float("inf"))
    st.load(xc, vprev)
    t = time_graph(st, steps, warmup)
    return {"workload": wc.name, "levels": 2, "dtype": dtype, "patches": st.np, "fine_nodes": st.nf,
            "network": "753-512-512-375", "indicator": True, "theta": None, "ms_per_step": t["ms"],
            "median_ms": t["median_ms"], "patches_per_s": st.np / (t["ms"] * 1e-3),
            "fine_dof_per_s": 4 * st.nf / (t["ms"] * 1e-3)}


def paper_network_params(n_in, hidden, n_out, depth=8, seed=0):
    """Seeded parameters of the paper's network form: N(0, 1/fan_in) weights,
    batch-normalisation gamma, beta and statistics near identity, the output
    layer scaled down (a small correction)."""
    rng = np.random.default_rng(seed)
    dims = [n_in] + [hidden] * depth + [n_out]
    Ws = [rng.standard_normal((dims[i], dims[i + 1])) / np.sqrt(dims[i]) for i in range(depth + 1)]
    Ws[-1] *= 0.05
    ga = [1.0 + 0.1 * rng.standard_normal(hidden) for _ in range(depth)]
    be = [0.05 * rng.standard_normal(hidden) for _ in range(depth)]
    mu = [0.05 * rng.standard_normal(hidden) for _ in range(depth)]
    sd = [np.exp(0.1 * rng.standard_normal(hidden)) for _ in range(depth)]
    return Ws, ga, be, mu, sd


def run_paper_network(steps, warmup):
    """The large channel's step with the paper's network form (240 inputs, 8
    hidden layers of width 750 with folded batch normalisation and skip
    connections, 81 outputs; BF16), indicator evaluated (threshold infinite),
    seeded parameters; and the network's forward alone in TFLOP/s."""
    import dnnmg_synth as syn
    from paper_2307_14837_amd import _lib as L
    from paper_2307_14837_amd import stepper

    w = syn.cfg5()
    inp = syn.step_inputs(w, seed=0)
    ps = paper_network_params(240, 750, 81)
    st = stepper.CorrectionStep(w.box, w.ns, ps, dtype="bf16", network="paper", indicator=True,
                                theta=float("inf"))
    st.load(inp.xc, inp.vprev)
    t = time_graph(st, steps, warmup)
    st.step()
    tf = time_kernel(lambda: L.dnnmg_deepnet_forward(st.deep, st.np, st.X, st.ldx, st.Y), 10)
    useful = 2 * (240 * 750 + 7 * 750 * 750 + 750 * 81) * st.np
    return {"workload": w.name, "network": "paper form 240-750x8-81 (batch norm folded, skip connections)",
            "dtype": "bf16", "indicator": True, "theta": None, "ms_per_step": t["ms"], "median_ms": t["median_ms"],
            "patches_per_s": st.np / (t["ms"] * 1e-3), "forward_ms": tf,
            "forward_tflops": useful / (tf * 1e-3) / 1e12,
            "forward_frac_of_bf16_peak": useful / (tf * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS}


def step_kernel_times(st, reps=20):
    """Each launch of the headline step timed alone on the step's own buffers
    (after one step, so every input holds step data): ms per launch."""
    from paper_2307_14837_amd import _lib as L

    box, ns = st.box, st.ns
    st.step()
    k = {
        "prolong_residual_b": lambda: L.dnnmg_prolong_residual_b(box, ns, st.xc, st.b, st.xt, st.r),
        "gather_forward": lambda: L.dnnmg_patch_gather_forward(box, st.net, st.xt, st.r, st.Y, st.shift,
                                                              st.inv_scale),
        "scatter": lambda: L.dnnmg_scatter_avg(box, st.Y, st.xcorr, vbase=st.xt),
        # the indicator's residual with the next right-hand side (b in place:
        # repeated calls leave the same b and r)
        "residual_rhs_b_indicator": lambda: L.dnnmg_residual_rhs_b(box, ns, st.xcorr, st.b, st.r2, st.ws_res,
                                                                   b_save=st.b_prev),
        "norm2_pair": lambda: L.dnnmg_norm2_pair_f64(st.r, st.r2, st.norms, st.ws_norm),
        "fallback_skipped": lambda: L.dnnmg_fallback_b(box, ns, st.xt, st.b_prev, st.norms, st.xcorr, st.ws_fb,
                                                       theta=st.theta, sweeps=st.fallback_sweeps,
                                                       flag_out=st.fell_back),
        "rhs_if_skipped": lambda: L.dnnmg_rhs_if(box, ns, st.xcorr, st.b, st.fell_back),
        "restrict": lambda: L.dnnmg_restrict(box, st.b, st.bc),
    }
    return {name: time_kernel(fn, reps) for name, fn in k.items()}


def roofline_of(kernel_ms, st, w):
    """Roofline object of the step's dominant launch (the largest of
    step_kernel_times), from the algorithmic counts per fine node of
    flops.ALG_*."""
    from paper_2307_14837_amd import flops

    name = max(kernel_ms, key=kernel_ms.get)
    t = kernel_ms[name]
    nf, npch = st.nf, st.np
    if name == "gather_forward":
        flop = flops.mlp_flops_per_patch(w.hidden) * npch
        peak = FP8_MFMA_PEAK_TFLOPS if st.dtype == 2 else BF16_MFMA_PEAK_TFLOPS
        return {"kernel": "dnnmg_patch_gather_forward", "bound": "mfma", "achieved": flop / (t * 1e-3) / 1e12,
                "peak": peak, "unit": "TFLOP/s", "frac": flop / (t * 1e-3) / 1e12 / peak,
                "traffic": traffic_from_profile("dnnmg_patch_gather_forward", w.name),
                "avg_launch_ms": t, "flop_per_launch": flop}
    per_node = {"residual_rhs_b_indicator": flops.ALG_RESIDUAL_RHS_B_GENERAL_PER_NODE,
                "prolong_residual_b": flops.ALG_PROLONG_RESIDUAL_B_PER_NODE}
    if name in per_node:
        flop = per_node[name] * nf
        entry = {"residual_rhs_b_indicator": "dnnmg_residual_rhs_b",
                 "prolong_residual_b": "dnnmg_prolong_residual_b"}[name]
        ach = flop / (t * 1e-3) / 1e12
        return {"kernel": entry, "bound": "alu", "achieved": ach, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP32_VALU_PEAK_TFLOPS, "traffic": traffic_from_profile(entry, w.name),
                "avg_launch_ms": t, "flop_per_launch": flop}
    nbytes = flops.BYTES_PER_FINE_NODE.get(name, 0) * nf
    ach = nbytes / (t * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "avg_launch_ms": t}


def accuracy(w, dtype, ref):
    """rel-L2 of one GPU step (seeded inputs and weights, indicator evaluated,
    fallback not taken) against the FP64 oracle reference of the same step."""
    st, inp = build_step(w, dtype, indicator=True, theta=float("inf"))
    out = st.run_numpy(inp.xc, inp.vprev)
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    tol = {"fp32": 1e-5, "bf16": 2e-2, "fp8": 5e-2}[dtype]
    res = {"xt": rel(out["xt"], ref["xt"]), "r": rel(out["r"], ref["r"]), "d": rel(out["d"], ref["d"]),
           "bc": rel(out["bc"], ref["bc"]), "eta_gpu": out["eta"], "eta_oracle": ref["eta"], "tol_d_bc": tol}
    res["within_tol"] = bool(res["r"] <= 1e-5 and res["d"] <= tol and res["bc"] <= tol)
    return res


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
    t = time_graph(bs, steps, warmup)
    npch, nf = bs.plan.n_patches, bs.plan.n_fine
    return {"workload": "cfg3_32_periodic_boxes", "boxes": len(boxes), "patches": npch, "fine_nodes": nf,
            "dtype": dtype, "fused_batched": True,
            "autotuned": {"patches_per_tile": ppt, "grid": grid,
                          "extension": "tiled" if bs.plan.scatter_form() == 2 else "per node"},
            "ms_per_step": t["ms"], "median_ms": t["median_ms"], "patches_per_s": npch / (t["ms"] * 1e-3),
            "fine_dof_per_s": 4 * nf / (t["ms"] * 1e-3)}


def run_per_box_plain(dtype, steps, warmup):
    """The same 32 boxes as separate plain steps (unfused gather, FP32 network),
    all 32 captured in one HIP graph."""
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

    t = time_graph(All(), steps, warmup)
    npch = sum(b.n_patches for b in boxes)
    nf = sum(b.n_fine for b in boxes)
    return {"workload": "cfg3_32_periodic_boxes", "boxes": len(boxes), "patches": npch, "dtype": dtype,
            "fused_batched": False, "ms_per_step": t["ms"], "patches_per_s": npch / (t["ms"] * 1e-3),
            "fine_dof_per_s": 4 * nf / (t["ms"] * 1e-3)}


def run_training(steps):
    """One AdamW step of the patch network at the training batch size
    (65,536 patches, width 256, BF16 compute, FP32 master weights)."""
    import torch

    import dnnmg_synth as syn
    from paper_2307_14837_amd import flops, train

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
    fl = 3 * flops.mlp_flops_per_patch(H) * n  # forward + backward (about 2x forward)
    return {"workload": "training_batch_65536_width256",
            "dtype": "bf16 forward and backward products, fp32 accumulation and master weights",
            "ms_per_step": ms, "patches_per_s": n / (ms * 1e-3), "approx_tflops": fl / (ms * 1e-3) / 1e12}


def run_coarse_step():
    """The GPU coarse step (Newton, FGMRES(16), one coupled patch-Vanka step
    as preconditioner) on the large channel's coarse mesh (128x32x32 cells,
    562 k unknowns): b^L = R Rhs(v0) of the channel start velocity, from the
    coarse start with its Dirichlet data; eager and graph-replayed times and
    the residual norms of the four Newton steps."""
    import time

    import torch

    import dnnmg_synth as syn
    from paper_2307_14837_amd import _lib as L

    w = syn.cfg5()
    box, ns = w.box, w.ns
    vf, vc = syn.channel_initial(box, seed=0)
    mask, vals = syn.channel_dirichlet(box, fine=False)
    F = torch.zeros(4 * box.n_fine, dtype=torch.float32, device="cuda")
    L.dnnmg_rhs(box, ns, torch.as_tensor(vf.astype(np.float32).ravel()).cuda(), F)
    b = torch.zeros(4 * box.n_coarse, dtype=torch.float64, device="cuda")
    L.dnnmg_restrict(box, F, b)
    b.masked_fill_(torch.as_tensor(mask.ravel()).cuda(), 0.0)
    x0 = np.zeros((4, box.n_coarse))
    x0[:3] = vc
    start = torch.as_tensor(np.where(mask, vals, x0).ravel()).cuda()
    o = L.coarse_opts(newton_its=4)
    ws = torch.empty(L.coarse_workspace_bytes(box, o), dtype=torch.uint8, device="cuda")
    res = torch.zeros(o.newton_its + 1, dtype=torch.float64, device="cuda")
    x = start.clone()
    L.dnnmg_coarse_solve(box, ns, b, x, o, ws, res)
    torch.cuda.synchronize()
    x.copy_(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L.dnnmg_coarse_solve(box, ns, b, x, o, ws, res)
    torch.cuda.synchronize()
    eager = time.perf_counter() - t0
    g = L.capture_graph(lambda: L.dnnmg_coarse_solve(box, ns, b, x, o, ws, res,
                                                     stream=torch.cuda.current_stream()))
    times = []
    for _ in range(3):
        x.copy_(start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.replay(torch.cuda.current_stream())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return {"workload": "coarse_step_channel_128x32x32", "unknowns": 4 * box.n_coarse,
            "method": "4 Newton steps, FGMRES(16) each, one coupled patch-Vanka step as preconditioner, "
                      "matrix-free Jacobian products",
            "ms_eager": eager * 1e3, "ms_graph": min(times) * 1e3,
            "residual_norms": [float(v) for v in res.cpu().numpy()]}


def q2_step(dtype="fp8", hidden=512, seed=0):
    """The correction step on the paper's discretisation (Q2/Q2 elements on
    curved hexahedra) for the large channel's mesh: 128 x 32 x 32 fine Q2
    elements (the patches), 1,085,825 nodes, interior nodes displaced
    smoothly by up to 0.15 element sizes; seeded network weights; indicator
    evaluated."""
    import dnnmg_synth as syn
    from paper_2307_14837_amd import stepper

    w = syn.cfg5()
    X = syn.distorted_coords(w.box, amp=0.15, seed=seed)
    inp = syn.step_inputs(w, seed=seed)
    params = syn.mlp_params(165, hidden, 81, seed=seed)
    st = stepper.Q2CorrectionStep(w.box, w.ns, X, params, dtype=dtype, indicator=True)
    st.load(inp.xc, inp.vprev)
    return w, st


def run_q2_step(steps, warmup, with_oracle=True):
    """Graph replays of the Q2 correction step (each replay's right-hand side
    feeds the next one's residual) and each launch timed alone; with_oracle:
    also the accuracy of one step against the FP64 Q2 oracle."""
    from paper_2307_14837_amd import _lib as L
    from paper_2307_14837_amd import flops

    w, st = q2_step()
    t = time_graph(st, steps, warmup)
    box, ns = st.box, st.ns
    k = {
        "q2_prolong": lambda: L.dnnmg_q2_prolong(box, st.xc, st.xt),
        "q2_residual_b": lambda: L.dnnmg_q2_residual_b(box, ns, st.coords, st.xt, st.b, st.r, ws=st.ws_q2),
        "gather_forward": lambda: L.dnnmg_patch_gather_forward_geom(box, st.net, st.geom, st.xt, st.r, st.Y),
        "scatter": lambda: L.dnnmg_scatter_avg(box, st.Y, st.xcorr, vbase=st.xt),
        "q2_residual_rhs_indicator": lambda: L.dnnmg_q2_residual_rhs(box, ns, st.coords, st.xcorr, st.b, st.r2,
                                                                     st.b2, ws=st.ws_q2),
        "norm2_pair": lambda: L.dnnmg_norm2_pair_f64(st.r, st.r2, st.norms, st.ws_norm),
        "q2_rhs": lambda: L.dnnmg_q2_rhs(box, ns, st.coords, st.xcorr, st.b, ws=st.ws_q2),
        "q2_restrict": lambda: L.dnnmg_q2_restrict(box, st.b, st.bc),
    }
    st.step()
    st.b2 = st.b.clone()  # the fused form's second output while timed alone
    kms = {name: time_kernel(fn, 10) for name, fn in k.items()}
    ne = st.np
    acc = q2_accuracy() if with_oracle else None
    res_flop = flops.q2_residual_flops_per_element() * ne
    rhs_flop = flops.q2_rhs_flops_per_element() * ne
    n = st.norms.cpu().numpy()
    return {"workload": "cfg5_channel_128x32x32_q2_curved", "elements": ne, "fine_nodes": st.nf,
            "discretisation": "Q2/Q2 on curved hexahedra (isoparametric), LPS with pi_h: Q2 -> Q1, "
                              "3x3x3 Gauss points, FP32",
            "network": "165-512-512-81 FP8 (seeded weights)", "dtype": "fp8", "indicator": True,
            "ms_per_step": t["ms"], "median_ms": t["median_ms"], "min_ms": t["min_ms"],
            "patches_per_s": ne / (t["ms"] * 1e-3), "kernel_ms": kms,
            "q2_residual": {"flop_per_element": flops.q2_residual_flops_per_element(),
                            "tflops": res_flop / (kms["q2_residual_b"] * 1e-3) / 1e12,
                            "frac_of_fp32_vector_peak": res_flop / (kms["q2_residual_b"] * 1e-3) / 1e12
                            / FP32_VALU_PEAK_TFLOPS,
                            "bytes_algorithmic_per_launch": flops.Q2_RESIDUAL_BYTES_PER_NODE * st.nf,
                            "traffic": traffic_from_profile("dnnmg_q2_residual_b", w.name)},
            "q2_rhs_tflops": rhs_flop / (kms["q2_rhs"] * 1e-3) / 1e12,
            "eta_last": float(np.sqrt(n[1] / n[0])) if n[0] > 0 else None,
            "accuracy_rel_l2": acc}


def q2_accuracy():
    """One Q2 step against the FP64 Q2 oracle on a curved channel of 64 x 16 x
    16 fine Q2 elements (the same mesh recipe; the oracle takes seconds there),
    seeded weights of width 512, indicator evaluated: rel-L2 of r, d, b^L and
    eta for the FP8 and BF16 networks."""
    import dnnmg_synth as syn
    from oracle import q2 as oq2
    from paper_2307_14837_amd import stepper

    w = syn.cfg2()
    X = syn.distorted_coords(w.box, amp=0.15, seed=0)
    inp = syn.step_inputs(w, seed=0)
    params = syn.mlp_params(165, 512, 81, seed=0)
    b = oq2.rhs(w.box, w.ns, X, np.asarray(inp.vprev, np.float32).astype(np.float64))
    p64 = [np.asarray(p, np.float32).astype(np.float64) for p in params]
    t0 = time.perf_counter()
    ref = oq2.correction_step(w.box, w.ns, X, p64, inp.xc, b, indicator=True, threads=CPU_WORKERS)
    t_oracle = time.perf_counter() - t0
    out = {"workload": "channel_64x16x16_q2_curved", "elements": w.box.n_patches,
           "oracle_step_s": t_oracle, "oracle_threads": CPU_WORKERS,
           "oracle_patches_per_s": w.box.n_patches / t_oracle}
    for dt in ("fp8", "bf16"):
        st = stepper.Q2CorrectionStep(w.box, w.ns, X, params, dtype=dt, indicator=True)
        g = st.run_numpy(inp.xc, inp.vprev)
        out[dt] = {"r": rel(g["r"], ref["r"]), "d": rel(g["d"], ref["d"]), "bc": rel(g["bc"], ref["bc"]),
                   "eta_gpu": g["eta"], "eta_oracle": ref["eta"]}
    return out


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def q2_profile(steps):
    """Only the Q2 step's graph replays (for rocprofv3 --kernel-trace)."""
    w, st = q2_step()
    st.capture()
    for _ in range(steps):
        st.replay()
    import torch

    torch.cuda.synchronize()
    print(json.dumps({"q2_profile": "cfg5_channel_128x32x32_q2_curved", "replays": steps}), flush=True)


def run_time_loop(w, params, shift, inv, steps=5):
    """Whole time steps of Algorithm 1 on the GPU, one graph each: the coarse
    problem (b^L the restriction of the previous step's fine Rhs) by the GPU
    coarse step (4 Newton steps), then the configured correction (FP8
    network, indicator at threshold 1, fallback), on the large channel."""
    import time

    import torch

    import dnnmg_synth as syn
    from paper_2307_14837_amd import _lib as L

    st, inp = build_step(w, "fp8", params, shift, inv, indicator=True, theta=1.0)
    mask, vals = syn.channel_dirichlet(w.box, fine=False)
    st.attach_coarse(L.coarse_opts(newton_its=4), (mask, vals))
    g = st.capture(full=True)
    torch.cuda.synchronize()
    ms, etas, fell, red = [], [], 0, []
    for _ in range(steps):
        t0 = time.perf_counter()
        g.replay(torch.cuda.current_stream())
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
        n = st.norms.cpu().numpy()
        etas.append(float(np.sqrt(n[1] / n[0])) if n[0] > 0 else 0.0)
        fell += int(st.fell_back.item())
        rc = st.c_res.cpu().numpy()
        red.append(float(rc[-1] / rc[0]) if rc[0] > 0 else 0.0)
    return {"workload": w.name + "_time_loop", "dtype": "fp8", "indicator": True, "theta": 1.0,
            "method": "coarse step on the GPU (4 Newton steps, FGMRES(16), one Vanka step as preconditioner) "
                      "+ the correction step, one graph per time step",
            "steps": steps, "ms_per_time_step_median": float(np.median(ms)), "eta": etas,
            "fallback_rate": fell / steps, "coarse_residual_reduction": red}


def run_config4(steps=200, train_steps=150, hidden=256, batch=65536, opt_steps=600):
    """The learned workload at its size: the channel of 48x12x12 coarse
    cells (fine 96x24x24), `steps` teacher-forced steps of the plain method
    generated on the GPU (coarse and fine solves by the GPU coarse step),
    BF16 training at width 256 and batch 65,536 on steps 1..150 with the
    library's kernels, and the relative velocity error of eq. (relerrors) on
    the held-out steps 151..200: DNN-MG against the prolongated coarse
    solution."""
    import time

    import torch

    import dnnmg_synth as syn
    from paper_2307_14837_amd import _lib as L
    from paper_2307_14837_amd import stepper, train

    w = syn.cfg4()
    box, ns = w.box, w.ns
    vf, vc = syn.channel_initial(box, amp=0.3, seed=0)
    cb = syn.BoxSpec(tuple(n // 2 for n in box.n), box.len, box.periodic_mask, box.dirichlet_mask)
    fbc, cbc = syn.channel_dirichlet(box, True), syn.channel_dirichlet(cb, True)
    xc0 = np.zeros((4, box.n_coarse))
    xc0[:3] = vc
    log = lambda m: print("[bench]   " + m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    xcs, vbar, _, norms = train.teacher_forced(box, ns, vf, xc0, steps, fbc, cbc, log=log)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    npch = box.n_patches
    t0 = time.perf_counter()
    X = train.gather_inputs(box, ns, [xcs[n].cpu().numpy() for n in range(train_steps)],
                            [vbar[n].cpu().numpy() for n in range(train_steps)], L.F32).view(train_steps * npch, -1)
    T = train.gather_targets(box, xcs[:train_steps], vbar[1:train_steps + 1])
    shift, inv = train.standardisation(X)
    Z = torch.zeros_like(X, dtype=torch.bfloat16)
    Z[:, :L.N_IN] = ((X[:, :L.N_IN] - shift) * inv).to(torch.bfloat16)
    del X
    t_scale = float(T.double().std().item())
    Tn = T / t_scale
    tr = train.PatchTrainer(train._init_params(hidden, 0), dtype="bf16", lr=1e-3, max_batch=batch)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    rows = train_steps * npch
    losses = []
    for it in range(opt_steps):
        idx = torch.randint(0, rows, (batch,), device="cuda", generator=g)
        tr.step(Z[idx].contiguous().view(-1), Tn[idx].contiguous().view(-1), batch)
        if it % 100 == 0 or it == opt_steps - 1:
            losses.append(tr.loss(batch))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    st = stepper.CorrectionStep(box, ns, tr.params(target_scale=t_scale), dtype="bf16",
                                shift=shift.cpu().numpy(), inv_scale=inv.cpu().numpy())
    e_plain, e_net = [], []
    for n in range(train_steps + 1, steps + 1):
        out = st.run_numpy(xcs[n - 1].cpu().numpy(), vbar[n - 1].cpu().numpy())
        ref = vbar[n].cpu().numpy().astype(np.float64)
        nrm = np.linalg.norm(ref)
        e_plain.append(np.linalg.norm(out["xt"][:3] - ref) / nrm)
        e_net.append(np.linalg.norm(out["vcorr"] - ref) / nrm)
    # the paper's network form (8 hidden layers of width 512, batch
    # normalisation with batch statistics, skip connections; its Sec. 4.2
    # inputs) on the same data, trained with torch autograd in FP32 and run
    # folded in the library's deep forward (BF16) inside the correction step
    t1 = time.perf_counter()
    Xp = train.paper_inputs(box, ns, xcs[:train_steps], vbar[:train_steps])
    p_shift, p_inv = train.standardisation(Xp, 240)
    Xp[:, :240] = (Xp[:, :240] - p_shift) * p_inv
    pparams, _, _, ploss = train.train_paper_network(Xp, T, hidden=512, depth=8, steps=400, batch=16384)
    del Xp
    torch.cuda.synchronize()
    t_paper = time.perf_counter() - t1
    stp = stepper.CorrectionStep(box, ns, pparams, dtype="bf16", network="paper", shift=p_shift.cpu().numpy(),
                                 inv_scale=p_inv.cpu().numpy())
    e_paper = []
    for n in range(train_steps + 1, steps + 1):
        out = stp.run_numpy(xcs[n - 1].cpu().numpy(), vbar[n - 1].cpu().numpy())
        ref = vbar[n].cpu().numpy().astype(np.float64)
        e_paper.append(np.linalg.norm(out["vcorr"] - ref) / np.linalg.norm(ref))
    fine_red = [float(f[-1] / f[0]) for _, f in norms if f[0] > 0]
    return {"workload": "cfg4_channel_48x12x12_learned", "steps": steps, "train_steps": train_steps,
            "held_out": [train_steps + 1, steps], "hidden": hidden, "batch": batch, "optimizer_steps": opt_steps,
            "data": "teacher-forced plain-method steps generated on the GPU (coarse and fine solves by the "
                    "GPU coarse step, 10 Newton steps each)",
            "fine_solve_residual_reduction_median": float(np.median(fine_red)),
            "seconds_data": t_data, "seconds_training": t_train,
            "training_loss": losses, "e_v_prolongation": float(np.mean(e_plain)),
            "e_v_dnnmg": float(np.mean(e_net)), "e_v_ratio": float(np.mean(e_net) / np.mean(e_plain)),
            "paper_network": {"form": "240-512x8-81, batch normalisation (batch statistics in training, folded "
                                      "for inference), skip connections; torch autograd FP32 training, 400 AdamW "
                                      "steps at batch 16,384; BF16 library forward",
                              "seconds_training": t_paper, "final_loss": ploss,
                              "e_v_dnnmg": float(np.mean(e_paper)),
                              "e_v_ratio": float(np.mean(e_paper) / np.mean(e_plain))}}


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
    st, inp = build_step(w, "bf16")
    st.step()
    torch.cuda.synchronize()
    nf, npch = st.nf, st.np
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
    t = time_kernel(lambda: L.dnnmg_prolong_residual_b(st.box, st.ns, st.xc, st.b, st.xt, st.r), reps)
    out["prolong_residual_b"] = {"ms": t, "TFLOP/s": flops.ALG_PROLONG_RESIDUAL_B_PER_NODE * nf / (t * 1e-3) / 1e12}
    t = time_kernel(lambda: L.dnnmg_rhs(st.box, st.ns, st.xcorr, st.b), reps)
    out["rhs"] = {"ms": t, "TFLOP/s": flops.ALG_RHS_PER_NODE * nf / (t * 1e-3) / 1e12}
    fl = flops.mlp_flops_per_patch(w.hidden) * npch
    for dtype in ("bf16", "fp8"):
        s2, _ = build_step(w, dtype)
        L.dnnmg_patch_gather(s2.box, s2.xt, s2.r, s2.X, s2.xdtype, 192, s2.shift, s2.inv_scale)
        for tp in (32, 64):
            t = time_kernel(lambda: L.dnnmg_patch_forward_tiles(s2.net, npch, s2.X, 192, s2.Y, tp), reps)
            out[f"forward_{dtype}_{tp}"] = {"ms": t, "TFLOP/s": fl / (t * 1e-3) / 1e12}
    return out


def pmc_probe():
    """The headline step's indicator residual (general iterate against the
    carried right-hand side), prolongation + residual and fused gather + FP8
    network, three launches each on step data, then a plain device copy of
    PMC_COPY_MIB MiB, for counter runs.  The network has seeded weights (no
    training in this run): its correction is nonzero on every patch, as the
    trained network's is, so the residual kernels do the same work, and the
    network's work does not depend on its weights."""
    import torch

    import dnnmg_synth as syn
    from paper_2307_14837_amd import _lib as L

    w = syn.cfg5()
    # the step without the indicator fills every buffer the indicator's
    # residual reads, and launches none of the kernels counted below
    st, _ = build_step(w, "fp8")
    st.step()
    r2 = torch.empty_like(st.r)
    b_io, b_save = st.b.clone(), torch.empty_like(st.b)
    torch.cuda.synchronize()
    for _ in range(3):
        L.dnnmg_residual_b(st.box, st.ns, st.xcorr, st.b, r2, st.ws_res)
    for _ in range(3):
        L.dnnmg_residual_rhs_b(st.box, st.ns, st.xcorr, b_io, r2, st.ws_res, b_save=b_save)
    for _ in range(3):
        L.dnnmg_prolong_residual_b(st.box, st.ns, st.xc, st.b, st.xt, st.r)
    for _ in range(3):
        L.dnnmg_patch_gather_forward(st.box, st.net, st.xt, st.r, st.Y, st.shift, st.inv_scale)
    torch.cuda.synchronize()
    del st
    # the Q2 residual (element kernel + per-node sum) on the curved channel mesh
    _, q = q2_step()
    q.step()
    torch.cuda.synchronize()
    for _ in range(3):
        L.dnnmg_q2_residual_b(q.box, q.ns, q.coords, q.xt, q.b, q.r, ws=q.ws_q2)
    torch.cuda.synchronize()
    del q
    n = PMC_COPY_MIB * 2**20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": w.name, "copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "src_hash": {e: src_hash(*f) for e, f in ENTRY_SOURCES.items()}}), flush=True)


def profile_step(steps):
    """The headline step alone: distilled FP8 network, indicator at threshold
    1, `steps` graph replays (for rocprofv3 --kernel-trace --stats)."""
    import torch

    import dnnmg_synth as syn

    w = syn.cfg5()
    params, shift, inv, _ = distilled_network(w)
    st, _ = build_step(w, "fp8", params, shift, inv, indicator=True, theta=1.0)
    st.capture()
    for _ in range(steps):
        st.replay()
    torch.cuda.synchronize()
    print(json.dumps({"profile_step": w.name, "replays": steps, "fell_back_last": int(st.fell_back.item())}),
          flush=True)


def main():
    args = parse()
    if args.cpu_worker is not None:
        cpu_worker(args.cpu_worker)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.pmc_probe:
        pmc_probe()
        return
    if args.q2_step:
        q2_profile(args.steps)
        return
    if args.profile_training:
        print(json.dumps(run_training(args.steps)), flush=True)
        return
    if args.profile_paper_net:
        print(json.dumps(run_paper_network(args.steps, args.warmup)), flush=True)
        return
    if args.profile_levels:
        print(json.dumps(run_levels("fp8", args.steps, args.warmup)), flush=True)
        return
    if args.profile_batched:
        print(json.dumps(run_batched("bf16", args.steps, args.warmup)), flush=True)
        return
    if args.profile_step:
        profile_step(args.steps)
        return
    if args.scale_only:
        print(json.dumps({"kernels_at_scale": kernels_at_scale()}), flush=True)
        return

    import dnnmg_synth as syn

    # CPU leg first, before the GPU is touched: the oracle's throughput on the
    # host cores, and the FP64 references of the accuracy figures
    cpu, refs = None, {}
    if not args.no_cpu:
        print("[bench] CPU oracle baseline (1 core, then all cores)", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
        print("[bench] FP64 oracle references (large channel, 16,384-patch channel)", file=sys.stderr, flush=True)
        refs["cfg5"] = oracle_reference(syn.cfg5())
        refs["cfg2"] = oracle_reference(syn.cfg2())

    import torch

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    w = syn.cfg5()
    print(f"[bench] {w.name}: training the network on the plain fine correction", file=sys.stderr, flush=True)
    params, shift, inv, dinfo = distilled_network(w)
    print(f"[bench] headline: FP8 network + indicator (theta 1), {args.steps} graph replays", file=sys.stderr,
          flush=True)
    head, st, t = run_step(w, "fp8", args.steps, args.warmup, params, shift, inv, indicator=True, theta=1.0,
                           account=True)
    kernel_ms = step_kernel_times(st)
    roof = roofline_of(kernel_ms, st, w)
    out = {
        "metric": "DNN-MG correction step throughput (patches/s; fine DOF/s also given)",
        "value": head["patches_per_s"],
        "unit": "patches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "median_ms_per_step": head["median_ms"],
        "min_ms_per_step": head["min_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp8",
        "data": "synthetic",
        "config": {"workload": w.name, "patches": st.np, "fine_nodes": st.nf, "fine_dofs": 4 * st.nf,
                   "network": "165-512-512-81 tanh; E4M3 hidden product (per-tensor scales), BF16 input and "
                              "output layers, FP32 accumulation",
                   "network_weights": "trained on the GPU on the plain fine correction of 4 other seeded inputs",
                   "stencils": "FP32 (prolongation from FP64, restriction to FP64)",
                   "indicator": "eta = ||r(x_corr)|| / ||r(x~)|| in FP64, theta = 1, fallback = 4 "
                                "pressure-held patch-Vanka sweeps",
                   "time_loop": "each replay's right-hand side feeds the next replay's residual",
                   "parallelism": "1 GPU", "graph": "hipGraph replay of the whole step"},
        "fine_dof_per_s": head["fine_dof_per_s"],
        "indicator": head["indicator_stats"],
        "network_training": dinfo,
        "roofline": roof,
        "step_kernel_ms": kernel_ms,
        "wall_s_timed": t["wall_s"],
    }
    if not args.no_variants:
        print("[bench] variants", file=sys.stderr, flush=True)
        sv, wv = max(args.steps // 4, 10), max(args.warmup // 4, 3)
        c2 = syn.cfg2()
        variants = [
            run_step(w, "fp32", sv, wv, params, shift, inv, indicator=True, theta=1.0, account=True)[0],
            run_step(w, "bf16", sv, wv, params, shift, inv, indicator=True, theta=1.0, account=True)[0],
            run_step(w, "fp8", sv, wv, params, shift, inv)[0],
            run_levels("fp8", sv, wv),
            run_paper_network(sv, wv),
            run_step(c2, "bf16", args.steps, args.warmup)[0],
            run_step(c2, "fp32", args.steps, args.warmup)[0],
            run_batched("bf16", sv, wv),
            run_batched("fp32", sv, wv),
            run_per_box_plain("fp32", sv, wv),
            run_training(20),
            run_coarse_step(),
            run_time_loop(w, params, shift, inv),
            run_config4(),
            run_q2_step(sv, wv, with_oracle=not args.no_cpu),
        ]
        out["variants"] = variants
        print("[bench] kernels on the large channel", file=sys.stderr, flush=True)
        out["kernels_at_scale"] = kernels_at_scale()
    if refs:
        print("[bench] accuracy against the FP64 oracle", file=sys.stderr, flush=True)
        out["accuracy_rel_l2"] = {
            "note": "one step on seeded inputs and seeded N(0, 1/fan_in) weights, indicator evaluated",
            "cfg5_channel_128x32x32": {dt: accuracy(w, dt, refs["cfg5"]) for dt in ("fp32", "bf16", "fp8")},
            "cfg2_channel_64x16x16": {dt: accuracy(syn.cfg2(), dt, refs["cfg2"]) for dt in ("fp32", "bf16")},
            "oracle_seconds": {k: v["seconds"] for k, v in refs.items()},
        }
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
