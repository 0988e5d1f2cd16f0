"""Two-level prediction (J = 2; Sec. 4.2 patches of 4x4x4 fine cells, 125
nodes, 375 outputs) on the GPU against the FP64 oracle: dof map and valence
bit-exact, prolongation over two levels (and bit for bit the one-level
prolongation applied twice), its transpose in FP64, gather and extension on
125-node patches, the 753-H-H-375 network in FP32/BF16/FP8, and whole steps
with the indicator and the fallback."""
import numpy as np
import pytest
import torch

import dnnmg_synth as syn
from gpu_util import dev, f32, rel_l2, say, to_gpu

pytestmark = pytest.mark.gpu

BOXES = {
    "channel": syn.channel_box((4, 2, 2)),
    "periodic": syn.BoxSpec((4, 2, 2), (1.0, 0.6, 0.5), 7, 0),
    "mixed": syn.BoxSpec((2, 4, 2), (1.2, 0.8, 0.5), 2, syn.X_LO | syn.Z_HI),
    "chan_mid": syn.channel_box((12, 4, 4)),
}


@pytest.fixture(scope="module")
def L():
    import paper_2307_14837_amd as L

    assert torch.cuda.is_available()
    return L


def p32(params):
    return [np.asarray(p, np.float32).astype(np.float64) for p in params]


@pytest.mark.parametrize("name", list(BOXES))
def test_dofmap_levels_bit_exact(L, orc, name):
    box = BOXES[name]
    nf, _, npch = L.level_sizes(box, 2)
    m = torch.empty(npch * 125, dtype=torch.int32, device=dev())
    mult = torch.empty(nf, dtype=torch.uint8, device=dev())
    L.dnnmg_patch_dofmap_levels(box, 2, m, mult)
    torch.cuda.synchronize()
    rm, rmult = orc.dofmap_levels(box, 2)
    assert np.array_equal(m.cpu().numpy().reshape(npch, 125), rm)
    assert np.array_equal(mult.cpu().numpy(), rmult)


@pytest.mark.parametrize("name", list(BOXES))
def test_prolong_restrict_levels(L, orc, name):
    box = BOXES[name]
    say("two-level transfer", name)
    nf, nc, _ = L.level_sizes(box, 2)
    rng = np.random.default_rng(3)
    xc = rng.standard_normal((4, nc))
    xf = torch.empty(4 * nf, dtype=torch.float32, device=dev())
    L.dnnmg_prolong_levels(box, 2, to_gpu(xc.ravel()), xf)
    torch.cuda.synchronize()
    got = xf.cpu().numpy().reshape(4, nf)
    ref = orc.prolong_levels(box, 2, f32(xc).astype(np.float64))
    assert rel_l2(got, ref) <= 1e-7
    assert np.max(np.abs(got - ref)) <= 8 * 2.0 ** -24 * np.max(np.abs(ref))
    # the one-level prolongation applied twice gives the same bits
    box2 = L.level_box(box, 2)
    mid = torch.empty(4 * L.box_sizes(box)[0], dtype=torch.float32, device=dev())
    L.dnnmg_prolong(box, to_gpu(xc.ravel()), mid)
    two = torch.empty_like(xf)
    L.dnnmg_prolong(box2, mid.double(), two)
    torch.cuda.synchronize()
    assert torch.equal(two, xf)
    # transpose, FP64
    bf = f32(rng.standard_normal((4, nf)))
    bc = torch.empty(4 * nc, dtype=torch.float64, device=dev())
    L.dnnmg_restrict_levels(box, 2, to_gpu(bf.ravel()), bc)
    torch.cuda.synchronize()
    refb = orc.restrict_levels(box, 2, bf.astype(np.float64))
    assert rel_l2(bc.cpu().numpy().reshape(4, nc), refb) <= 1e-13


@pytest.mark.parametrize("name", list(BOXES))
@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_gather_scatter_levels(L, orc, name, dtype):
    box = BOXES[name]
    say("two-level gather/scatter", name, dtype)
    nf, _, npch = L.level_sizes(box, 2)
    rng = np.random.default_rng(5)
    x = f32(rng.standard_normal((4, nf)))
    r = f32(rng.standard_normal((4, nf)) * 1e-2)
    sh = f32(rng.standard_normal(753) * 0.1)
    inv = f32(rng.uniform(0.5, 2.0, 753))
    dt = {"fp32": L.F32, "bf16": L.BF16}[dtype]
    X = torch.zeros(npch * 768, dtype=torch.float32 if dtype == "fp32" else torch.bfloat16, device=dev())
    L.dnnmg_patch_gather_levels(box, 2, to_gpu(x.ravel()), to_gpu(r.ravel()), X, dt, 768, to_gpu(sh), to_gpu(inv))
    torch.cuda.synchronize()
    got = X.float().cpu().numpy().reshape(npch, 768)
    ref = orc.gather_levels(box, 2, x.astype(np.float64), r.astype(np.float64), sh.astype(np.float64),
                            inv.astype(np.float64))
    assert np.all(got[:, 753:] == 0.0)
    if dtype == "fp32":
        assert np.max(np.abs(got[:, :753] - ref)) <= 4 * 2.0 ** -24 * (np.abs(ref) + 1.0).max()
    else:
        # BF16 rounding of each value (relative half-ulp 2^-9)
        assert np.all(np.abs(got[:, :753] - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-30)
        assert rel_l2(got[:, :753], ref) <= 4e-3
    Y = f32(rng.standard_normal((npch, 375)))
    d = torch.empty(3 * nf, dtype=torch.float32, device=dev())
    L.dnnmg_scatter_avg_levels(box, 2, to_gpu(Y.ravel()), d)
    xb = to_gpu(x.ravel())
    dx = torch.empty(4 * nf, dtype=torch.float32, device=dev())
    L.dnnmg_scatter_avg_levels(box, 2, to_gpu(Y.ravel()), dx, vbase=xb)
    torch.cuda.synchronize()
    refd = orc.scatter_levels(box, 2, Y.astype(np.float64))
    assert rel_l2(d.cpu().numpy().reshape(3, nf), refd) <= 1e-6
    gx = dx.cpu().numpy().reshape(4, nf)
    assert np.array_equal(gx[3], x[3])
    assert rel_l2(gx[:3], x[:3].astype(np.float64) + refd) <= 1e-6


@pytest.mark.parametrize("dtype,H,n,tol", [("fp32", 256, 33, 1e-5), ("fp32", 256, 1000, 1e-5),
                                           ("bf16", 256, 17, 2e-2), ("bf16", 512, 1000, 2e-2),
                                           ("bf16", 512, 4099, 2e-2), ("fp8", 512, 1000, 5e-2)])
def test_mlp_levels_forward(L, orc, dtype, H, n, tol):
    from paper_2307_14837_amd.stepper import DTYPES

    say("753-H-375 network", dtype, H, n)
    params = syn.mlp_params(753, H, 375, seed=7, bias_scale=0.1)
    dt = DTYPES[dtype]
    prep = L.mlp_prepare(dt, H, [to_gpu(f32(params[2 * l])) for l in range(3)],
                         [to_gpu(f32(params[2 * l + 1])) for l in range(3)], n_in=753, n_out=375)
    rng = np.random.default_rng(8)
    X = f32(rng.standard_normal((n, 753)))
    Xp = np.zeros((n, 768), np.float32)
    Xp[:, :753] = X
    Xg = to_gpu(Xp.ravel())
    if dt != L.F32:
        Xg = Xg.to(torch.bfloat16)
    Y = torch.full((n * 375,), float("nan"), dtype=torch.float32, device=dev())
    L.dnnmg_patch_forward(prep.net, n, Xg, 768, Y)
    torch.cuda.synchronize()
    ref = orc.mlp_forward(X.astype(np.float64), *p32(params))
    e = rel_l2(Y.cpu().numpy().reshape(n, 375), ref)
    say(f"  rel-L2 {e:.2e}")
    assert e <= tol


@pytest.mark.parametrize("name,dtype,tol", [("channel", "fp32", 1e-4), ("periodic", "fp32", 1e-4),
                                            ("chan_mid", "bf16", 2e-2), ("chan_mid", "fp8", 5e-2)])
def test_step_levels_vs_oracle(orc, name, dtype, tol):
    """One J = 2 correction step (indicator evaluated, no fallback) against the
    oracle's chain with levels = 2."""
    from paper_2307_14837_amd import stepper

    box = BOXES[name]
    say("two-level step", name, dtype)
    ns = syn.NSParams(1e-3, 0.005) if "chan" in name else syn.NSParams(1e-3, 0.01)
    import oracle as O

    nf = O.fine_nodes(O.level_box(box, 2))
    rng = np.random.default_rng(9)
    w = syn.Workload("w", box, ns, 256, dtype, "channel" if "chan" in name else "fourier")
    inp = syn.step_inputs(w, seed=9)
    xc = inp.xc
    vprev = O.prolong_levels(box, 2, xc)[:3] + 0.05 * rng.standard_normal((3, nf))
    vprev[:, O.dirichlet_flags(O.level_box(box, 2)).astype(bool)] = O.prolong_levels(box, 2, xc)[:3][
        :, O.dirichlet_flags(O.level_box(box, 2)).astype(bool)]
    H = 512 if dtype == "fp8" else 256
    params = syn.mlp_params(753, H, 375, seed=10)
    params[4] = params[4] * 0.05
    st = stepper.CorrectionStep(box, ns, params, dtype=dtype, levels=2, indicator=True, theta=float("inf"))
    out = st.run_numpy(xc, vprev)
    ref = orc.correction_step(box, ns, p32(params), xc, out["vprev32"], levels=2, indicator=True,
                              theta=float("inf"))
    assert rel_l2(out["xt"], ref["xt"]) <= 1e-7
    er = rel_l2(out["r"], ref["r"])
    say(f"  r rel-L2 {er:.2e}")
    assert er <= 1e-5
    for key in ("Y", "d", "bc"):
        e = rel_l2(out[key], ref[key])
        say(f"  {key} rel-L2 {e:.2e}")
        assert e <= tol, key
    assert abs(out["eta"] - ref["eta"]) <= max(tol, 1e-5) * ref["eta"]


def test_step_levels_fallback(orc):
    """theta = 0 on a J = 2 channel step: the plain fine correction (patch
    sweeps on level L + 2) replaces the network's."""
    from paper_2307_14837_amd import stepper

    box = BOXES["channel"]
    ns = syn.NSParams(1e-3, 0.005)
    inp = syn.step_inputs(syn.Workload("w", box, ns, 256, "fp32", "channel"), seed=11)
    import oracle as O

    vprev = O.prolong_levels(box, 2, inp.xc)[:3]
    params = syn.mlp_params(753, 256, 375, seed=12)
    st = stepper.CorrectionStep(box, ns, params, dtype="fp32", levels=2, indicator=True, theta=0.0,
                                fallback_sweeps=3)
    out = st.run_numpy(inp.xc, vprev)
    ref = orc.correction_step(box, ns, p32(params), inp.xc, out["vprev32"], levels=2, indicator=True,
                              theta=0.0, fallback_sweeps=3)
    assert out["fell_back"] == ref["fell_back"] == 1
    for key in ("vcorr", "bc"):
        e = rel_l2(out[key], ref[key])
        say(f"  fallback {key} rel-L2 {e:.2e}")
        assert e <= 1e-4, key


@pytest.mark.parametrize("name", list(BOXES))
def test_prolong_residual_b_levels(L, orc, name):
    """Two-level prolongation fused with the level L + 2 residual against
    b = Rhs(v_prev): x~ is dnnmg_prolong_levels' bit for bit, and r is the
    oracle's Crank-Nicolson residual at x~ (whose local projection terms
    vanish, x~ being the patch interpolant of level L + 1)."""
    box = BOXES[name]
    say("two-level prolongation + residual", name)
    ns = syn.NSParams(1e-3, 0.01)
    fb = L.level_box(box, 2)
    nf, nc, _ = L.level_sizes(box, 2)
    rng = np.random.default_rng(31)
    xc = rng.standard_normal((4, nc))
    vp = f32(rng.standard_normal((3, nf)))
    xcg, vpg = to_gpu(xc.ravel()), to_gpu(vp.ravel())
    new = lambda: torch.full((4 * nf,), float("nan"), dtype=torch.float32, device=dev())
    xt0 = new()
    L.dnnmg_prolong_levels(box, 2, xcg, xt0)
    b = new()
    L.dnnmg_rhs(fb, ns, vpg, b)
    ws = torch.empty(L.prolong_residual_b_levels_workspace_bytes(box, 2), dtype=torch.uint8, device=dev())
    assert ws.numel() == (8 * 4 * L.level_sizes(box, 1)[0] + 255) // 256 * 256
    xt, r = new(), new()
    L.dnnmg_prolong_residual_b_levels(box, 2, ns, xcg, b, xt, r, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(xt0, xt)
    ref = orc.residual(fb, ns, xt.cpu().numpy().reshape(4, -1).astype(np.float64), vp.astype(np.float64))
    e = rel_l2(r.cpu().numpy().reshape(4, -1), ref)
    say(f"  rel-L2 {e:.2e}")
    assert e <= 1e-5
    with pytest.raises(L.DnnmgError):
        L.dnnmg_prolong_residual_b_levels(box, 2, ns, xcg, b, xt, b, ws=ws)
    with pytest.raises(L.DnnmgError):
        L.dnnmg_prolong_residual_b_levels(box, 2, ns, xcg, b, xt, r, ws=ws[:8])
