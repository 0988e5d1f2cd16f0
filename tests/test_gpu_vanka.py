"""Plain fine-level correction (patch-Vanka sweeps) on the GPU against the oracle."""
import numpy as np
import pytest
import torch

import dnnmg_synth as syn
from gpu_util import dev, f32, rel_l2, say, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_2307_14837_amd as L

    assert torch.cuda.is_available()
    return L


CASES = {
    "cfg1": (syn.cfg1().box, syn.cfg1().ns),
    "chan_small": (syn.channel_box((4, 2, 2)), syn.NSParams(1e-3, 0.005)),
    "mixed": (syn.BoxSpec((6, 4, 2), (1.2, 0.8, 0.5), 1, syn.Y_LO | syn.Y_HI | syn.Z_HI),
              syn.NSParams(0.01, 0.01, 0.05, 0.1)),
}


def inputs(box, orc, seed):
    rng = np.random.default_rng(seed)
    xc = rng.standard_normal((4, box.n_coarse))
    x = orc.prolong(box, xc)
    vp = x[:3] + 0.2 * rng.standard_normal((3, box.n_fine))
    dmask = syn.boundary_mask(box, True)
    vp[:, dmask] = x[:3, dmask]
    return f32(x), f32(vp)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("sweeps", [1, 3])
@pytest.mark.parametrize("coupled", [False, True])
def test_vanka_sweeps_match_oracle(L, orc, name, sweeps, coupled):
    box, ns = CASES[name]
    say("vanka", name, "sweeps", sweeps, "coupled" if coupled else "pressure held")
    x, vp = inputs(box, orc, 3)
    omega = 1.0 if not coupled else 0.7
    xg = to_gpu(x.ravel().copy())
    ws = torch.empty(L.vanka_workspace_bytes(box), dtype=torch.uint8, device=dev())
    L.dnnmg_vanka_sweeps(box, ns, xg, to_gpu(vp.ravel()), ws, sweeps=sweeps, omega=omega, coupled=coupled)
    got = xg.cpu().numpy().reshape(4, -1).astype(np.float64)
    ref = x.astype(np.float64)
    for _ in range(sweeps):
        ref = orc.vanka_sweep(box, ns, ref, vp.astype(np.float64), omega=omega, coupled=coupled)
    e = rel_l2(got - x, ref - x)
    say(f"  correction rel-L2 {e:.2e}")
    assert e <= 2e-3 if coupled else e <= 1e-4
    if not coupled:
        assert np.array_equal(got[3], x[3].astype(np.float64))
        r0 = np.linalg.norm(orc.residual(box, ns, x.astype(np.float64), vp.astype(np.float64))[:3])
        r1 = np.linalg.norm(orc.residual(box, ns, got, vp.astype(np.float64))[:3])
        say(f"  momentum residual {r0:.3e} -> {r1:.3e}")
        assert r1 < r0 / 3.0 ** sweeps


@pytest.mark.parametrize("name", list(CASES))
def test_fallback_against_rhs_matches_oracle(L, orc, name):
    """The fallback whose sweep residuals are r = b - A(x), b = Rhs(v_prev):
    taken (theta = 0), it gives the oracle's pressure-held sweeps from x~; not
    taken (theta = inf), x_corr is left as it is."""
    box, ns = CASES[name]
    say("fallback against b", name)
    x, vp = inputs(box, orc, 5)
    nf = box.n_fine
    xt = to_gpu(x.ravel())
    b = torch.empty(4 * nf, dtype=torch.float32, device=dev())
    L.dnnmg_rhs(box, ns, to_gpu(vp.ravel()), b)
    ws = torch.empty(L.fallback_workspace_bytes(box), dtype=torch.uint8, device=dev())
    norms = torch.tensor([1.0, 1.0], dtype=torch.float64, device=dev())
    flag = torch.zeros(1, dtype=torch.int32, device=dev())
    keep = to_gpu(f32(np.full(4 * nf, 7.0)))
    L.dnnmg_fallback_b(box, ns, xt, b, norms, keep, ws, theta=float("inf"), sweeps=2, flag_out=flag)
    torch.cuda.synchronize()
    assert flag.item() == 0 and torch.all(keep == 7.0)
    xcorr = torch.empty(4 * nf, dtype=torch.float32, device=dev())
    L.dnnmg_fallback_b(box, ns, xt, b, norms, xcorr, ws, theta=0.0, sweeps=2, flag_out=flag)
    torch.cuda.synchronize()
    assert flag.item() == 1
    got = xcorr.cpu().numpy().reshape(4, -1).astype(np.float64)
    ref = x.astype(np.float64)
    for _ in range(2):
        ref = orc.vanka_sweep(box, ns, ref, vp.astype(np.float64), omega=1.0, coupled=False)
    e = rel_l2(got - x, ref - x)
    say(f"  correction rel-L2 {e:.2e}")
    assert e <= 1e-4


NORM_CASES = [(0.0, 0.0), (0.0, 1.0), (1.0, 0.5), (1.0, 2.0), (1.0, float("nan")), (0.0, float("nan"))]


@pytest.mark.parametrize("theta", [1.0, float("inf")])
def test_indicator_flag_decisions(L, orc, theta):
    """The device decision of the residual indicator equals the oracle's on
    hand-set norms: a zero reference residual (0/0 reads as eta = 0), a NaN
    corrected residual, and theta = inf, which never falls back."""
    box, ns = CASES[list(CASES)[0]]
    nf = box.n_fine
    xt = to_gpu(f32(np.full(4 * nf, 3.0)))
    b = torch.zeros(4 * nf, dtype=torch.float32, device=dev())
    ws = torch.empty(L.fallback_workspace_bytes(box), dtype=torch.uint8, device=dev())
    flag = torch.full((1,), -1, dtype=torch.int32, device=dev())
    for n0, n1 in NORM_CASES:
        say("indicator flag", theta, n0, n1)
        norms = torch.tensor([n0, n1], dtype=torch.float64, device=dev())
        xcorr = to_gpu(f32(np.full(4 * nf, 7.0)))
        L.dnnmg_fallback_b(box, ns, xt, b, norms, xcorr, ws, theta=theta, sweeps=0, flag_out=flag)
        torch.cuda.synchronize()
        want = orc.fallback_taken(n0, n1, theta)
        assert flag.item() == want, (n0, n1, theta)
        # zero sweeps: a taken fallback leaves x~ itself, else x_corr is kept
        assert torch.all(xcorr == (3.0 if want else 7.0))
