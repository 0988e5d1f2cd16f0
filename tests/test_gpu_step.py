"""End-to-end correction step on the GPU against the oracle chain, and the
HIP-graph replay against eager execution."""
import numpy as np
import pytest
import torch

import dnnmg_synth as syn
from gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stepper():
    from paper_2307_14837_amd import stepper

    assert torch.cuda.is_available()
    return stepper


def p32(params):
    return [np.asarray(p, np.float32).astype(np.float64) for p in params]


@pytest.mark.parametrize("dtype,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_step_cfg1(stepper, orc, dtype, tol):
    w = syn.cfg1()
    say("step cfg1", dtype)
    inp = syn.step_inputs(w, seed=0)
    params = syn.mlp_params(165, w.hidden, 81, seed=0)
    # theta = inf: the indicator is evaluated but the fallback never taken
    st = stepper.CorrectionStep(w.box, w.ns, params, dtype=dtype, indicator=True, theta=float("inf"))
    out = st.run_numpy(inp.xc, inp.vprev)
    ref = orc.correction_step(w.box, w.ns, p32(params), inp.xc, out["vprev32"], indicator=True,
                              theta=float("inf"))
    assert rel_l2(out["xt"], ref["xt"]) <= 1e-7
    assert rel_l2(out["r"], ref["r"]) <= 1e-5
    for key in ("Y", "d", "vcorr", "b", "bc"):
        e = rel_l2(out[key], ref[key])
        say(f"  {key} rel-L2 {e:.2e}")
        assert e <= tol, key
    assert abs(out["eta"] - ref["eta"]) <= max(tol, 1e-5) * ref["eta"]


def test_step_cfg2_bf16(stepper, orc):
    w = syn.cfg2()
    say("step cfg2 bf16")
    inp = syn.step_inputs(w, seed=0)
    params = syn.mlp_params(165, w.hidden, 81, seed=0)
    st = stepper.CorrectionStep(w.box, w.ns, params, dtype="bf16")
    out = st.run_numpy(inp.xc, inp.vprev)
    ref = orc.correction_step(w.box, w.ns, p32(params), inp.xc, out["vprev32"])
    assert rel_l2(out["r"], ref["r"]) <= 1e-5
    for key in ("d", "b", "bc"):
        e = rel_l2(out[key], ref[key])
        say(f"  {key} rel-L2 {e:.2e}")
        assert e <= 2e-2, key


def test_graph_replay_matches_eager(stepper):
    w = syn.cfg1()
    say("graph replay cfg1")
    inp = syn.step_inputs(w, seed=1)
    params = syn.mlp_params(165, w.hidden, 81, seed=1)
    st = stepper.CorrectionStep(w.box, w.ns, params, dtype="bf16", indicator=True)
    eager = st.run_numpy(inp.xc, inp.vprev)
    st.capture()
    for rep in range(4):
        st.load(inp.xc, inp.vprev)  # the step carries the right-hand side: start again
        st.bc.zero_()
        st.xcorr.zero_()
        torch.cuda.synchronize()
        st.replay()
        torch.cuda.synchronize()
        assert np.array_equal(st.bc.cpu().numpy().reshape(4, -1), eager["bc"]), rep
        assert np.array_equal(st.xcorr.cpu().numpy().reshape(4, -1)[:3], eager["vcorr"].astype(np.float32))


def test_carried_rhs_graph_and_vprev_form(stepper):
    """A step that carries the right-hand side (r = b - A(x~), b from the
    previous step) matches the step built from v_prev up to FP32 rounding,
    and its graph replays match the eager step when b is reset in between."""
    w = syn.cfg2()
    say("carried rhs cfg2")
    inp = syn.step_inputs(w, seed=3)
    params = syn.mlp_params(165, w.hidden, 81, seed=3)
    a = stepper.CorrectionStep(w.box, w.ns, params, dtype="fp32", carry_rhs=True)
    b = stepper.CorrectionStep(w.box, w.ns, params, dtype="fp32", carry_rhs=False)
    oa, ob = a.run_numpy(inp.xc, inp.vprev), b.run_numpy(inp.xc, inp.vprev)
    assert np.array_equal(oa["xt"], ob["xt"])
    for key in ("r", "d", "b", "bc"):
        e = rel_l2(oa[key], ob[key])
        say(f"  {key} rel-L2 {e:.2e}")
        assert e <= 1e-5, key
    st = stepper.CorrectionStep(w.box, w.ns, params, dtype="bf16")
    assert st.carry_rhs
    eager = st.run_numpy(inp.xc, inp.vprev)
    st.load(inp.xc, inp.vprev)
    b0 = st.b.clone()
    st.capture()
    for rep in range(3):
        st.b.copy_(b0)
        st.bc.zero_()
        torch.cuda.synchronize()
        st.replay()
        torch.cuda.synchronize()
        assert np.array_equal(st.bc.cpu().numpy().reshape(4, -1), eager["bc"]), rep
        assert np.array_equal(st.r.cpu().numpy().reshape(4, -1), eager["r"].astype(np.float32)), rep


@pytest.mark.parametrize("mode", ["never", "always", "nan_weights", "huge_weights"])
def test_indicator_fallback(stepper, orc, mode):
    """Residual-indicator fallback forced from the host: theta = inf (never),
    theta = 0 (always), NaN weights and weights scaled by 1e3 (both must fall
    back, decided on the device)."""
    w = syn.cfg1()
    say("fallback", mode)
    inp = syn.step_inputs(w, seed=2)
    params = syn.mlp_params(165, w.hidden, 81, seed=2)
    theta = {"never": float("inf"), "always": 0.0}.get(mode, 1.0)
    if mode == "nan_weights":
        params[4] = params[4].copy(); params[4][0, 0] = np.nan
    if mode == "huge_weights":
        params[4] = params[4] * 1e3
    st = stepper.CorrectionStep(w.box, w.ns, params, dtype="fp32", indicator=True, theta=theta,
                                fallback_sweeps=3)
    out = st.run_numpy(inp.xc, inp.vprev)
    ref = orc.correction_step(w.box, w.ns, p32(params), inp.xc, out["vprev32"], indicator=True,
                              theta=theta, fallback_sweeps=3)
    assert out["fell_back"] == ref["fell_back"] == (0 if mode == "never" else 1)
    assert np.all(np.isfinite(out["vcorr"])) and np.all(np.isfinite(out["bc"]))
    tol = 1e-4 if out["fell_back"] else 1e-5
    for key in ("vcorr", "bc"):
        e = rel_l2(out[key], ref[key])
        say(f"  {key} rel-L2 {e:.2e}")
        assert e <= tol, key
    if mode != "never":
        # the plain correction lowers the momentum residual of x~
        r_fb = orc.residual(w.box, w.ns, np.concatenate([out["vcorr"], out["xt"][3:4]]), out["vprev32"])
        assert np.linalg.norm(r_fb[:3]) < np.linalg.norm(ref["r"][:3])
