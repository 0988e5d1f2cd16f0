"""GPU coarse step (Newton, FGMRES, multigrid with patch-Vanka smoothing)
against the FP64 oracle: its Jacobian-vector product, its preconditioner,
a manufactured solution and the oracle's own Newton solve of a time step's
coarse problem (Alg. 1; Sec. 2.4)."""
import numpy as np
import pytest
import torch

import dnnmg_synth as syn
from gpu_util import dev, rel_l2, say, to_gpu

pytestmark = pytest.mark.gpu

NS = syn.NSParams(1e-3, 0.005)


@pytest.fixture(scope="module")
def L():
    import paper_2307_14837_amd as L

    assert torch.cuda.is_available()
    return L


def obox(box):
    """The box whose fine mesh is the coarse mesh of `box` (how the oracle
    evaluates the coarse operator)."""
    return syn.BoxSpec(tuple(n // 2 for n in box.n), box.len, box.periodic_mask, box.dirichlet_mask)


def A_of(orc, ob, y):
    """A(y) on the fine mesh of ob (the oracle residual with no explicit
    part is -A(y); Dirichlet velocity rows zero)."""
    return -orc.residual(ob, NS, y, np.zeros((3, ob.n_fine)))


def jv_oracle(orc, ob, x, z):
    """J(x) z by central differences of the FP64 oracle operator."""
    h = 1e-6 * (np.sqrt(np.mean(x * x)) + 1e-6) / np.sqrt(np.mean(z * z))
    return (A_of(orc, ob, x + h * z) - A_of(orc, ob, x - h * z)) / (2 * h)


def manufactured(box, seed):
    """A state x* on the coarse mesh of `box` (the channel's divergence-free
    start velocity with its Dirichlet data, a smooth pressure) and a start
    x0 that agrees with x* on the Dirichlet velocity entries."""
    rng = np.random.default_rng(seed)
    _, vc = syn.channel_initial(box, seed=seed)
    mask, vals = syn.channel_dirichlet(box, fine=False)
    p = syn.node_coords(box, fine=False)
    xs = np.zeros((4, box.n_coarse))
    xs[:3] = vc
    xs[3] = 0.3 * np.cos(np.pi * p[0] / box.len[0]) + 0.1 * p[1]
    xs = np.where(mask, vals, xs)
    x0 = xs + 0.05 * rng.standard_normal(xs.shape)
    x0 = np.where(mask, xs, x0)
    return xs, x0, mask


def random_dir(box, seed, mask):
    z = np.random.default_rng(seed).standard_normal((4, box.n_coarse))
    return np.where(mask, 0.0, z)


def workspace(L, box, opts):
    return torch.empty(L.coarse_workspace_bytes(box, opts), dtype=torch.uint8, device=dev())


BOXES = {"chan16x8x8": syn.channel_box((16, 8, 8)), "chan8x4x4": syn.channel_box((8, 4, 4))}


def test_coarse_levels(L):
    o = L.coarse_opts(levels=0)
    assert L.coarse_levels(syn.channel_box((16, 8, 8)), o) == 2
    assert L.coarse_levels(syn.channel_box((128, 32, 32)), o) == 4
    assert L.coarse_levels(syn.channel_box((128, 32, 32)), L.coarse_opts(levels=2)) == 2
    with pytest.raises(L.DnnmgError):
        L.coarse_levels(syn.channel_box((9, 4, 4)), o)
    with pytest.raises(L.DnnmgError):
        L.coarse_levels(syn.channel_box((8, 4, 4)), L.coarse_opts(krylov_dim=L.COARSE_MAX_KRYLOV + 1))


@pytest.mark.parametrize("name", list(BOXES))
def test_coarse_jv_matches_oracle(L, orc, name):
    """The matrix-free FP32 Jacobian-vector product against central
    differences of the FP64 oracle operator."""
    box = BOXES[name]
    ob = obox(box)
    xs, x0, mask = manufactured(box, 1)
    z = random_dir(box, 2, mask)
    o = L.coarse_opts()
    ws = workspace(L, box, o)
    xg = to_gpu(x0.astype(np.float32))
    zg = to_gpu(z.astype(np.float32))
    w = torch.zeros_like(xg)
    say("coarse jv", name)
    L.dnnmg_coarse_jv(box, NS, xg, zg, w, o, ws)
    torch.cuda.synchronize()
    ref = jv_oracle(orc, ob, x0.astype(np.float32).astype(np.float64), z.astype(np.float32).astype(np.float64))
    got = w.cpu().numpy().astype(np.float64).reshape(4, -1)
    errs = [rel_l2(got[f], ref[f]) for f in range(4)]
    say("  rel-L2 per field", errs)
    assert max(errs[:3]) <= 2e-3 and errs[3] <= 2e-2
    assert np.all(got[:3][mask[:3]] == 0.0)


def patch_dofs(ob, M):
    """Global dofs [u, v, w, p] x local node a + 3b + 9c of patch M of the
    fine mesh of ob (non-periodic)."""
    nx, ny, _ = ob.fine_shape
    I, J, K = M % ob.n[0], (M // ob.n[0]) % ob.n[1], M // (ob.n[0] * ob.n[1])
    idx = np.array([(2 * I + a) + nx * ((2 * J + b) + ny * (2 * K + c))
                    for c in range(3) for b in range(3) for a in range(3)])
    return np.concatenate([f * ob.n_fine + idx for f in range(4)])


def vanka_step(orc, ob, x, d, omega):
    """One linear coupled patch-Vanka step from z = 0 on the fine mesh of ob:
    z = omega * mu (.) sum_P A_P^-1 d_P with the oracle's local matrices A_P
    (linearised at the velocity of x), Dirichlet velocities zero."""
    nf = ob.n_fine
    acc, cnt = np.zeros(4 * nf), np.zeros(4 * nf)
    d = np.asarray(d, dtype=np.float64).ravel()
    for M in range(ob.n_patches):
        P = patch_dofs(ob, M)
        acc[P] += orc.dense_solve(orc.vanka_matrix(ob, NS, x[:3], M), d[P])
        cnt[P] += 1
    z = omega * acc / np.maximum(cnt, 1)
    dm = orc.dirichlet_flags(ob).astype(bool)
    for f in range(3):
        z[f * nf:(f + 1) * nf][dm] = 0.0
    return z.reshape(4, nf)


def inject(ob, x):
    """The coarse-node values of a field on the fine mesh of ob."""
    nx, ny, nz = ob.fine_shape
    return x.reshape(4, nz, ny, nx)[:, ::2, ::2, ::2].reshape(4, -1)


@pytest.mark.parametrize("name", list(BOXES))
@pytest.mark.parametrize("levels", [1, 2])
def test_coarse_vcycle_matches_oracle(L, orc, name, levels):
    """The preconditioner: levels = 1 is one coupled patch-Vanka step on the
    coarse mesh; levels = 2 adds the coarse-grid correction (defect
    restricted with P^T, one Vanka step on the halved mesh linearised at
    the injected iterate, prolongated), rebuilt here from oracle pieces
    (local matrices, FD64 Jacobian products, transfers)."""
    box = BOXES[name]
    ob = obox(box)
    xs, x0, mask = manufactured(box, 3)
    x0 = x0.astype(np.float32).astype(np.float64)
    s = (1e-3 * random_dir(box, 4, mask)).astype(np.float32).astype(np.float64)
    omega = 0.8
    o = L.coarse_opts(levels=levels, pre_sweeps=1, post_sweeps=0, coarsest_sweeps=1, omega=omega)
    if L.coarse_levels(box, o) < levels:
        pytest.skip("the halved mesh is below 4 cells per axis")
    ws = workspace(L, box, o)
    z = torch.zeros(4 * box.n_coarse, dtype=torch.float32, device=dev())
    L.dnnmg_coarse_vcycle(box, NS, to_gpu(x0.astype(np.float32)), to_gpu(s.astype(np.float32)), z, o, ws)
    torch.cuda.synchronize()
    got = z.cpu().numpy().astype(np.float64).reshape(4, -1)
    ref = vanka_step(orc, ob, x0, s, omega)
    if levels == 2:
        ob1 = obox(ob)
        d = s - jv_oracle(orc, ob, x0, ref)
        s1 = orc.restrict(ob, d)
        s1[:3][orc.dirichlet_flags(ob1).astype(bool)[None, :].repeat(3, 0)] = 0.0
        z1 = vanka_step(orc, ob1, inject(ob, x0), s1, omega)
        ref = ref + orc.prolong(ob, z1)
    errs = [rel_l2(got[f], ref[f]) for f in range(4)]
    say("coarse v-cycle", name, "levels", levels, "rel-L2 per field", errs)
    assert np.all(np.isfinite(got)) and np.all(got[:3][mask[:3]] == 0.0)
    assert max(errs) <= 1e-2


@pytest.mark.parametrize("name", list(BOXES))
def test_coarse_solve_manufactured(L, orc, name):
    """b = A(x*) by the oracle; the GPU solve from a perturbed start returns
    x* to FP32 accuracy, and the oracle's residual at its result is small."""
    box = BOXES[name]
    ob = obox(box)
    xs, x0, mask = manufactured(box, 5)
    b = A_of(orc, ob, xs)
    o = L.coarse_opts(newton_its=10)
    ws = workspace(L, box, o)
    x = to_gpu(x0)
    res = torch.zeros(o.newton_its + 1, dtype=torch.float64, device=dev())
    L.dnnmg_coarse_solve(box, NS, to_gpu(b), x, o, ws, res)
    torch.cuda.synchronize()
    got = x.cpu().numpy().reshape(4, -1)
    rn = res.cpu().numpy()
    say("coarse solve", name, "residual norms", rn)
    ev, ep = rel_l2(got[:3], xs[:3]), rel_l2(got[3], xs[3])
    rr = np.linalg.norm(b - A_of(orc, ob, got)) / np.linalg.norm(b)
    say("  rel-L2 velocity", ev, "pressure", ep, "oracle residual / ||b||", rr)
    assert np.all(got[:3][mask[:3]] == x0[:3][mask[:3]])
    assert rn[-1] <= 1e-3 * rn[0]
    assert ev <= 1e-3 and ep <= 1e-2
    assert rr <= 1e-4


def test_coarse_solve_time_step_matches_oracle_newton(L, orc):
    """The coarse problem of one time step (Alg. 1): b^L = R Rhs_fine(v) with
    the Dirichlet velocity rows zero, solved by the oracle's Newton method
    (FD Jacobian, sparse LU, rtol 1e-10) and on the GPU from the same start."""
    from oracle.solve import NewtonSolver

    box = syn.channel_box((8, 4, 4))
    ob = obox(box)
    vf, vc = syn.channel_initial(box, seed=7)
    F = orc.rhs(box, NS, vf)
    bL = orc.restrict(box, F)
    mask, vals = syn.channel_dirichlet(box, fine=False)
    bL[:3][mask[:3]] = 0.0
    x0 = np.zeros((4, box.n_coarse))
    x0[:3] = vc
    x0 = np.where(mask, vals, x0)
    zero = np.zeros((3, ob.n_fine))
    ref, its = NewtonSolver(ob, NS).solve(lambda z: bL + orc.residual(ob, NS, z, zero), x0)
    say("oracle Newton iterations", its)
    o = L.coarse_opts(newton_its=10)
    ws = workspace(L, box, o)
    x = to_gpu(x0)
    res = torch.zeros(o.newton_its + 1, dtype=torch.float64, device=dev())
    L.dnnmg_coarse_solve(box, NS, to_gpu(bL), x, o, ws, res)
    torch.cuda.synchronize()
    got = x.cpu().numpy().reshape(4, -1)
    ev, ep = rel_l2(got[:3], ref[:3]), rel_l2(got[3], ref[3])
    say("coarse time step: residual norms", res.cpu().numpy(), "rel-L2 velocity", ev, "pressure", ep)
    assert ev <= 1e-3 and ep <= 1e-2


def test_coarse_solve_graph_replays(L, orc):
    """The solve recorded into a graph (dnnmg_graph_capture_*) and replayed
    three times from the same start, with eager work between the replays,
    gives the eager result bit for bit each time."""
    box = BOXES["chan16x8x8"]
    ob = obox(box)
    xs, x0, _ = manufactured(box, 9)
    b = to_gpu(A_of(orc, ob, xs))
    o = L.coarse_opts(newton_its=2)
    ws = workspace(L, box, o)
    start = to_gpu(x0)
    x = start.clone()
    L.dnnmg_coarse_solve(box, NS, b, x, o, ws)
    torch.cuda.synchronize()
    eager = x.cpu().numpy()
    xg = start.clone()

    def run():
        L.dnnmg_coarse_solve(box, NS, b, xg, o, ws, stream=torch.cuda.current_stream())

    g = L.capture_graph(run)
    for _ in range(3):
        xg.copy_(start)
        torch.cuda.synchronize()
        g.replay(torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert np.array_equal(xg.cpu().numpy(), eager)


def test_gpu_time_step_matches_oracle(L, orc):
    """A whole time step of Algorithm 1 on the GPU (stepper.time_step: coarse
    problem b^L = R Rhs(v_prev) solved by the GPU coarse step, then the
    correction with an FP32 network), recorded into one graph and replayed
    for two steps, against the oracle: its Newton solve of the same coarse
    problem and its FP64 correction step, chained."""
    from oracle.solve import NewtonSolver

    from paper_2307_14837_amd import stepper

    box = syn.channel_box((8, 4, 4))
    ob = obox(box)
    vf, vc = syn.channel_initial(box, seed=11)
    mask, vals = syn.channel_dirichlet(box, fine=False)
    xc0 = np.where(mask, vals, np.concatenate([vc, np.zeros((1, box.n_coarse))]))
    params = syn.mlp_params(165, 64, 81, seed=3, bias_scale=0.1)
    params[4] = params[4] * 0.01  # a small correction, as a trained network gives
    st = stepper.CorrectionStep(box, NS, params, dtype="fp32")
    st.load(xc0, vf)
    st.attach_coarse(L.coarse_opts(newton_its=10), (mask, vals))
    g = st.capture(full=True)  # the eager warm-up is time step 1
    torch.cuda.synchronize()
    got1 = st.xcorr.cpu().numpy().reshape(4, -1)[:3].astype(np.float64)
    g.replay(torch.cuda.current_stream())  # time step 2
    torch.cuda.synchronize()
    got2 = st.xcorr.cpu().numpy().reshape(4, -1)[:3].astype(np.float64)
    p64 = [np.asarray(p, np.float32).astype(np.float64) for p in params]
    zero = np.zeros((3, ob.n_fine))
    x, vprev = xc0, vf
    for n, got in ((1, got1), (2, got2)):
        bL = orc.restrict(box, orc.rhs(box, NS, vprev))
        bL[:3][mask[:3]] = 0.0
        x = np.where(mask, vals, x)
        x, _ = NewtonSolver(ob, NS).solve(lambda z: bL + orc.residual(ob, NS, z, zero), x)
        ref = orc.correction_step(box, NS, p64, x, vprev)
        err = rel_l2(got, ref["vcorr"])
        say(f"time step {n}: corrected velocity rel-L2 {err:.2e}")
        assert err <= 1e-4
        vprev = ref["vcorr"]
