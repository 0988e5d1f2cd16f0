"""The paper's discretisation on the GPU (Q2/Q2 elements on curved hexahedra,
LPS with pi_h: Q2 -> Q1; Sec. 2.2 eq. (disc:ns), Sec. 2.3 eq.
(4cranknicholson3), (stabparams); the Q2 transfer of Algorithm 1) against the
FP64 Q2 oracle, element by element on seeded distorted channel meshes,
through the C ABI.

Tolerances: the kernels evaluate every element integral in FP32 from FP32
fields and FP32 offsets of the node positions (the positions themselves are
FP64), so each term carries a relative error of a few FP32 roundings (about
1e-7 of its size).  r = b - A(x) is compared per field against ||b|| + ||r||
(the terms it is the difference of) with 1e-5; the transfer operators, which
round once to FP32 (prolongation) or accumulate FP32 inputs in FP64
(restriction), are compared at 2e-7 and 1e-13.
"""
import numpy as np
import pytest
import torch

import dnnmg_synth as syn
from gpu_util import f32, rel_l2, say, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2307_14837_amd import _lib

    assert torch.cuda.is_available()
    return _lib


@pytest.fixture(scope="module")
def q2():
    from oracle import q2 as mod

    mod.lib()
    return mod


BOXES = [((4, 2, 2), 1), ((5, 3, 2), 2), ((8, 4, 4), 3)]
NS = syn.NSParams(1e-3, 0.005)


def channel_case(n, seed, amp=0.15):
    box = syn.channel_box(n)
    X = syn.distorted_coords(box, amp=amp, seed=seed)
    rng = np.random.default_rng(100 + seed)
    w = syn.Workload("q2", box, NS, 32, "fp32", "channel")
    base = syn.step_inputs(w, seed=seed)
    # a fine iterate near the channel state: vprev plus noise, pressure from
    # the coarse ramp at the even nodes spread by noise
    x = np.zeros((4, box.n_fine))
    x[:3] = base.vprev + 0.05 * rng.standard_normal((3, box.n_fine))
    x[3] = 0.4 * (box.len[0] - syn.node_coords(box, True)[0]) + 0.05 * rng.standard_normal(box.n_fine)
    return box, X, base, x


def field_err(a, ref, scale):
    return [np.linalg.norm(a[f] - ref[f]) / max(scale[f], 1e-30) for f in range(ref.shape[0])]


@pytest.mark.parametrize("n,seed", BOXES)
def test_q2_residual_matches_oracle(L, q2, n, seed):
    box, X, base, x = channel_case(n, seed)
    say("q2 residual", n, "seed", seed)
    x32 = f32(x)
    rng = np.random.default_rng(seed)
    for kind in ("rhs", "random"):
        b = q2.rhs(box, NS, X, f32(base.vprev)) if kind == "rhs" else rng.standard_normal((4, box.n_fine))
        b32 = f32(b)
        r = torch.zeros(4 * box.n_fine, dtype=torch.float32, device="cuda")
        L.dnnmg_q2_residual_b(box, NS, to_gpu(X.ravel()), to_gpu(x32.ravel()), to_gpu(b32.ravel()), r)
        torch.cuda.synchronize()
        rg = r.cpu().numpy().reshape(4, -1).astype(np.float64)
        ro = q2.residual_b(box, NS, X, x32.astype(np.float64), b32.astype(np.float64))
        scale = [np.linalg.norm(b32[f]) + np.linalg.norm(ro[f]) for f in range(4)]
        err = field_err(rg, ro, scale)
        say(f"  b={kind}: per-field error / (|b| + |r|) {['%.1e' % e for e in err]}, "
            f"rel-L2 {[('%.1e' % rel_l2(rg[f], ro[f])) for f in range(4)]}")
        assert max(err) <= 1e-5
        dm = syn.boundary_mask(box, fine=True)
        assert np.all(rg[:3, dm] == 0.0)


@pytest.mark.parametrize("n,seed", BOXES[:2])
def test_q2_rhs_matches_oracle(L, q2, n, seed):
    box, X, base, x = channel_case(n, seed)
    say("q2 rhs", n)
    v32 = f32(x[:3])
    fm32 = f32(np.random.default_rng(seed + 7).standard_normal((3, box.n_fine)))
    for fm in (None, fm32):
        b = torch.zeros(4 * box.n_fine, dtype=torch.float32, device="cuda")
        L.dnnmg_q2_rhs(box, NS, to_gpu(X.ravel()), to_gpu(v32.ravel()), b,
                       fmid=None if fm is None else to_gpu(fm.ravel()))
        torch.cuda.synchronize()
        bg = b.cpu().numpy().reshape(4, -1).astype(np.float64)
        bo = q2.rhs(box, NS, X, v32.astype(np.float64), None if fm is None else fm.astype(np.float64))
        err = [rel_l2(bg[f], bo[f]) for f in range(3)]
        say(f"  fmid={'yes' if fm is not None else 'no'}: rel-L2 {['%.1e' % e for e in err]}")
        assert max(err) <= 1e-6
        assert np.all(bg[3] == 0.0)


@pytest.mark.parametrize("n", [(4, 2, 2), (8, 4, 6), (16, 8, 4)])
def test_q2_transfer_matches_oracle(L, q2, n):
    box = syn.channel_box(n)
    say("q2 transfer", n)
    rng = np.random.default_rng(sum(n))
    xc = rng.standard_normal((4, box.n_coarse))
    xf = torch.zeros(4 * box.n_fine, dtype=torch.float32, device="cuda")
    L.dnnmg_q2_prolong(box, to_gpu(xc.ravel()), xf)
    bf = f32(rng.standard_normal((4, box.n_fine)))
    bc = torch.zeros(4 * box.n_coarse, dtype=torch.float64, device="cuda")
    L.dnnmg_q2_restrict(box, to_gpu(bf.ravel()), bc)
    torch.cuda.synchronize()
    po = q2.prolong(box, xc)
    pg = xf.cpu().numpy().reshape(4, -1).astype(np.float64)
    assert np.abs(pg - po).max() <= 2e-7 * np.abs(po).max()
    ro = q2.restrict(box, bf.astype(np.float64))
    rg = bc.cpu().numpy().reshape(4, -1)
    assert rel_l2(rg, ro) <= 1e-13


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_q2_gather_matches_oracle(L, q2, dtype):
    """Geometry inputs of the curved cells (once per mesh) and the gather with
    per-patch geometry against the oracle's element gather."""
    box, X, base, x = channel_case((4, 2, 2), 5)
    say("q2 gather", dtype)
    rng = np.random.default_rng(9)
    r = f32(rng.standard_normal((4, box.n_fine)))
    x32 = f32(x)
    shift = f32(rng.standard_normal(165))
    inv = f32(rng.uniform(0.5, 2.0, 165))
    geom = torch.zeros(3 * box.n_patches, dtype=torch.float32, device="cuda")
    L.dnnmg_q2_patch_features(box, to_gpu(X.ravel()), geom)
    ldx = 192
    tdt = torch.float32 if dtype == "fp32" else torch.bfloat16
    Xg = torch.full((box.n_patches * ldx,), 7.0, dtype=tdt, device="cuda")
    L.dnnmg_patch_gather_geom(box, geom, to_gpu(x32.ravel()), to_gpu(r.ravel()), Xg,
                              L.F32 if dtype == "fp32" else L.BF16, ldx, to_gpu(shift), to_gpu(inv))
    torch.cuda.synchronize()
    feat = q2.features(box, X)
    assert np.abs(geom.cpu().numpy().reshape(-1, 3) - feat).max() <= 1e-7 * np.abs(feat).max()
    G = Xg.float().cpu().numpy().reshape(box.n_patches, ldx).astype(np.float64)
    ref = q2.gather(box, X, x32.astype(np.float64), r.astype(np.float64), shift.astype(np.float64),
                    inv.astype(np.float64))
    tol = 1e-6 if dtype == "fp32" else 2 ** -8
    assert np.all(np.abs(G[:, :165] - ref) <= tol * np.maximum(np.abs(ref), 1.0))
    assert np.all(G[:, 165:] == 0.0)


def test_fused_gather_forward_geom_equals_separate(L):
    """The fused gather + network with per-patch geometry equals the
    separate gather and forward bit for bit (FP8 network, BF16 rows)."""
    from paper_2307_14837_amd import stepper

    box, X, base, x = channel_case((8, 4, 4), 6)
    params = syn.mlp_params(165, 256, 81, seed=4)
    st = stepper.Q2CorrectionStep(box, NS, X, params, dtype="fp8")
    st.load(base.xc, base.vprev)
    st.step()
    torch.cuda.synchronize()
    Y_fused = st.Y.clone()
    L.dnnmg_patch_gather_geom(box, st.geom, st.xt, st.r, st.X, L.BF16, st.ldx)
    L.dnnmg_patch_forward(st.net, st.np, st.X, st.ldx, st.Y)
    torch.cuda.synchronize()
    assert torch.equal(st.Y, Y_fused)


def p32(params):
    return [np.asarray(p, np.float32).astype(np.float64) for p in params]


@pytest.mark.parametrize("dtype,tol", [("fp32", 1e-5), ("bf16", 2e-2), ("fp8", 5e-2)])
def test_q2_step_matches_oracle(q2, dtype, tol):
    from paper_2307_14837_amd import stepper

    box = syn.channel_box((8, 4, 4))
    X = syn.distorted_coords(box, amp=0.15, seed=11)
    w = syn.Workload("q2", box, NS, 64, dtype, "channel")
    inp = syn.step_inputs(w, seed=11)
    params = syn.mlp_params(165, 128 if dtype == "fp8" else 64, 81, seed=2)
    say("q2 step", dtype)
    st = stepper.Q2CorrectionStep(box, NS, X, params, dtype=dtype, indicator=True)
    out = st.run_numpy(inp.xc, inp.vprev)
    vprev32 = f32(inp.vprev).astype(np.float64)
    b = q2.rhs(box, NS, X, vprev32)
    ref = q2.correction_step(box, NS, X, p32(params), inp.xc, b, indicator=True)
    assert rel_l2(out["xt"], ref["xt"]) <= 2e-7
    scale = [np.linalg.norm(b[f]) + np.linalg.norm(ref["r"][f]) for f in range(4)]
    assert max(field_err(out["r"], ref["r"], scale)) <= 1e-5
    for key in ("Y", "d", "vcorr", "b", "bc"):
        e = rel_l2(out[key], ref[key])
        say(f"  {key} rel-L2 {e:.2e}")
        assert e <= tol, key
    say(f"  eta gpu {out['eta']:.6f} oracle {ref['eta']:.6f}")
    assert abs(out["eta"] - ref["eta"]) <= max(tol, 1e-5) * ref["eta"]


def test_q2_step_reproducible_and_graph_replays(q2):
    from paper_2307_14837_amd import stepper

    box = syn.channel_box((8, 4, 4))
    X = syn.distorted_coords(box, amp=0.15, seed=12)
    w = syn.Workload("q2", box, NS, 64, "bf16", "channel")
    inp = syn.step_inputs(w, seed=12)
    params = syn.mlp_params(165, 64, 81, seed=3)
    say("q2 graph")
    st = stepper.Q2CorrectionStep(box, NS, X, params, dtype="bf16", indicator=True)
    st.load(inp.xc, inp.vprev)
    b0 = st.b.clone()
    st.step()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (st.r, st.xcorr, st.b, st.bc, st.norms)]
    # the same step again from the same right-hand side: bit for bit
    st.b.copy_(b0)
    st.step()
    torch.cuda.synchronize()
    for a, e in zip((st.r, st.xcorr, st.b, st.bc, st.norms), eager):
        assert torch.equal(a, e)
    st.b.copy_(b0)
    st.capture()  # one eager warm-up run, then the recording
    for rep in range(3):
        st.b.copy_(b0)
        torch.cuda.synchronize()
        st.replay()
        torch.cuda.synchronize()
        for a, e in zip((st.r, st.xcorr, st.b, st.bc, st.norms), eager):
            assert torch.equal(a, e), rep


def test_q2_residual_at_scale_matches_oracle(L, q2):
    """The residual kernel in the launch configuration of the large channel
    (128 x 32 x 32 fine Q2 elements, 1,085,825 nodes) against the oracle on
    the whole mesh."""
    box = syn.channel_box((128, 32, 32))
    X = syn.distorted_coords(box, amp=0.15, seed=21)
    w = syn.Workload("q2", box, NS, 32, "fp32", "channel")
    inp = syn.step_inputs(w, seed=21)
    say("q2 residual at scale: oracle prolongation and rhs")
    xt = q2.prolong(box, inp.xc)
    x32 = f32(xt)
    b32 = f32(q2.rhs(box, NS, X, f32(inp.vprev).astype(np.float64)))
    r = torch.zeros(4 * box.n_fine, dtype=torch.float32, device="cuda")
    L.dnnmg_q2_residual_b(box, NS, to_gpu(X.ravel()), to_gpu(x32.ravel()), to_gpu(b32.ravel()), r)
    torch.cuda.synchronize()
    rg = r.cpu().numpy().reshape(4, -1).astype(np.float64)
    say("q2 residual at scale: oracle residual")
    ro = q2.residual_b(box, NS, X, x32.astype(np.float64), b32.astype(np.float64))
    scale = [np.linalg.norm(b32[f]) + np.linalg.norm(ro[f]) for f in range(4)]
    err = field_err(rg, ro, scale)
    say(f"  per-field error / (|b| + |r|) {['%.1e' % e for e in err]}")
    assert max(err) <= 1e-5


@pytest.fixture(scope="module")
def dn():
    from oracle import deepnet

    return deepnet


@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_q2_paper_inputs_match_oracle(L, q2, dtype):
    """The 24 geometry features of curved cells (general form, from the 8
    vertices) and the paper-form gather on the Q2 elements against the
    oracle."""
    box, X, base, x = channel_case((4, 2, 2), 7, amp=0.2)
    say("q2 paper inputs", dtype)
    rng = np.random.default_rng(19)
    r = f32(rng.standard_normal((4, box.n_fine)))
    x32 = f32(x)
    shift = f32(rng.standard_normal(240))
    inv = f32(rng.uniform(0.5, 2.0, 240))
    geo = torch.zeros(24 * box.n_patches, dtype=torch.float32, device="cuda")
    L.dnnmg_q2_patch_features24(box, to_gpu(X.ravel()), geo)
    ldx = 256
    tdt = torch.float32 if dtype == "fp32" else torch.bfloat16
    Xg = torch.full((box.n_patches * ldx,), 7.0, dtype=tdt, device="cuda")
    L.dnnmg_patch_gather_paper_geom(box, geo, to_gpu(x32.ravel()), to_gpu(r.ravel()), Xg,
                                    L.F32 if dtype == "fp32" else L.BF16, ldx, to_gpu(shift), to_gpu(inv))
    torch.cuda.synchronize()
    ref = q2.paper_inputs(box, X, x32.astype(np.float64), r.astype(np.float64))
    g = geo.cpu().numpy().reshape(-1, 24)
    assert np.abs(g - ref[:, 216:]).max() <= 1e-6 * np.abs(ref[:, 216:]).max()
    # the curved cells' angles differ from the brick's pi/2
    assert np.abs(ref[:, 232:] - np.pi / 2).max() > 1e-3
    G = Xg.float().cpu().numpy().reshape(box.n_patches, ldx).astype(np.float64)
    z = (ref - shift.astype(np.float64)) * inv.astype(np.float64)
    tol = 2e-6 if dtype == "fp32" else 2 ** -8
    assert np.all(np.abs(G[:, :240] - z) <= tol * np.maximum(np.abs(z), 1.0))
    assert np.all(G[:, 240:] == 0.0)


@pytest.mark.parametrize("dtype,tol", [("fp32", 1e-4), ("bf16", 2e-2)])
def test_q2_step_paper_network_matches_oracle(q2, dn, dtype, tol):
    """The correction step on the paper's discretisation with the paper's
    network form (240-512x8-81, batch normalisation folded, skip
    connections) against the oracle's step."""
    from paper_2307_14837_amd import stepper

    box = syn.channel_box((8, 4, 4))
    X = syn.distorted_coords(box, amp=0.15, seed=13)
    w = syn.Workload("q2", box, NS, 64, dtype, "channel")
    inp = syn.step_inputs(w, seed=13)
    ps = dn.random_params(240, 512, 81, 8, seed=7)
    ps[0][-1] = ps[0][-1] * 0.05  # a modest correction
    say("q2 step, paper network", dtype)
    st = stepper.Q2CorrectionStep(box, NS, X, ps, dtype=dtype, indicator=True, network="paper")
    out = st.run_numpy(inp.xc, inp.vprev)
    b = q2.rhs(box, NS, X, f32(inp.vprev).astype(np.float64))
    r32 = [[np.asarray(a, np.float32).astype(np.float64) for a in group] for group in ps]
    ref = q2.correction_step(box, NS, X, r32, inp.xc, b, indicator=True, network="paper")
    for key in ("Y", "d", "b", "bc"):
        e = rel_l2(out[key], ref[key])
        say(f"  {key} rel-L2 {e:.2e}")
        assert e <= tol, key
    assert abs(out["eta"] - ref["eta"]) <= max(tol, 1e-5) * ref["eta"]


def test_q2_three_chained_steps_match_oracle_chain(q2):
    """Three Q2 steps in a row, each residual against the Rhs the previous
    step left (Algorithm 1's carried right-hand side), against the oracle's
    chain; the coarse solution is fixed, so the chain exercises the carried b
    and the network's dependence on it."""
    from paper_2307_14837_amd import stepper

    box = syn.channel_box((8, 4, 4))
    X = syn.distorted_coords(box, amp=0.15, seed=17)
    w = syn.Workload("q2", box, NS, 64, "fp32", "channel")
    inp = syn.step_inputs(w, seed=17)
    params = syn.mlp_params(165, 64, 81, seed=8)
    params[4] = params[4] * 0.1  # a modest correction
    st = stepper.Q2CorrectionStep(box, NS, X, params, dtype="fp32", indicator=True)
    st.load(inp.xc, inp.vprev)
    b = q2.rhs(box, NS, X, f32(inp.vprev).astype(np.float64))
    p64 = [np.asarray(p, np.float32).astype(np.float64) for p in params]
    for k in range(3):
        st.step()
        torch.cuda.synchronize()
        ref = q2.correction_step(box, NS, X, p64, inp.xc, b, indicator=True)
        bg = st.b.cpu().numpy().reshape(4, -1).astype(np.float64)
        bcg = st.bc.cpu().numpy().reshape(4, -1)
        e_b, e_bc = rel_l2(bg, ref["b"]), rel_l2(bcg, ref["bc"])
        say(f"  step {k}: b rel-L2 {e_b:.2e}, bc {e_bc:.2e}")
        assert e_b <= 1e-5 and e_bc <= 1e-5, k
        b = ref["b"]


def test_q2_residual_rhs_fused_matches_separate_and_oracle(L, q2):
    """The fused indicator residual + next right-hand side equals the two
    separate entry points (and the oracle), also in place (bnext = b)."""
    box, X, base, x = channel_case((5, 3, 2), 9)
    say("q2 fused residual + rhs")
    rng = np.random.default_rng(23)
    x32 = f32(x)
    b32 = f32(rng.standard_normal((4, box.n_fine)))
    Xg, xg, bg = to_gpu(X.ravel()), to_gpu(x32.ravel()), to_gpu(b32.ravel())
    nf4 = 4 * box.n_fine
    r_sep, b_sep = (torch.zeros(nf4, dtype=torch.float32, device="cuda") for _ in range(2))
    L.dnnmg_q2_residual_b(box, NS, Xg, xg, bg, r_sep)
    L.dnnmg_q2_rhs(box, NS, Xg, xg[:3 * box.n_fine].contiguous(), b_sep)
    r_f, bn_f = (torch.zeros(nf4, dtype=torch.float32, device="cuda") for _ in range(2))
    L.dnnmg_q2_residual_rhs(box, NS, Xg, xg, bg, r_f, bn_f)
    b_in = bg.clone()
    r_i = torch.zeros(nf4, dtype=torch.float32, device="cuda")
    L.dnnmg_q2_residual_rhs(box, NS, Xg, xg, b_in, r_i, b_in)  # in place
    torch.cuda.synchronize()
    assert torch.equal(r_f, r_sep)
    assert torch.equal(r_i, r_f) and torch.equal(b_in, bn_f)
    e = rel_l2(bn_f.cpu().numpy(), b_sep.cpu().numpy())
    say(f"  Rhs fused vs separate rel-L2 {e:.1e}")
    assert e <= 1e-6
    ref = q2.rhs(box, NS, X, x32[:3].astype(np.float64))
    assert rel_l2(bn_f.cpu().numpy().reshape(4, -1), ref) <= 1e-6
