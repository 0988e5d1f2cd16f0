"""Pins of the oracle's two-level prediction (J = 2, Sec. 4.2: patches of
4x4x4 fine cells, 125 nodes, 375 velocity outputs): each checked against
something other than the oracle itself (brute force, closed forms, a
Kronecker product of textbook 1-D matrices, adjointness, consistency)."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import dnnmg_synth as syn

BOXES = {
    "periodic": syn.BoxSpec((2, 4, 2), (1.0, 0.8, 0.6), 7, 0),
    "channel": syn.channel_box((3, 2, 2)),
    "mixed": syn.BoxSpec((2, 2, 4), (1.2, 0.7, 0.5), 1, syn.Y_LO | syn.Z_HI),
}


def lattice2(box):
    """Nodes per axis of the J = 2 lattice (4n cells per axis)."""
    return [4 * box.n[a] if (box.periodic_mask >> a) & 1 else 4 * box.n[a] + 1 for a in range(3)]


def node2(box, i, j, k):
    N = lattice2(box)
    c = [i, j, k]
    for a in range(3):
        if (box.periodic_mask >> a) & 1:
            c[a] %= N[a]
    return c[0] + N[0] * (c[1] + N[1] * c[2])


@pytest.mark.parametrize("name", list(BOXES))
def test_dofmap_levels_brute_force(orc, name):
    """Each patch's 125 nodes are the union of the vertex lists of its 64 fine
    cells, ordered by local coordinates; valences follow the closed form
    m = prod_a (2 if i_a = 0 mod 4 and the node is interior or the axis
    periodic, else 1) and sum to 125 N_p."""
    box = BOXES[name]
    m, mult = orc.dofmap_levels(box, 2)
    N = lattice2(box)
    for I, J, K in itertools.product(range(box.n[0]), range(box.n[1]), range(box.n[2])):
        M = I + box.n[0] * (J + box.n[1] * K)
        verts = {}
        for ci, cj, ck in itertools.product(range(4), repeat=3):
            for a, b, c in itertools.product(range(2), repeat=3):
                loc = (ci + a, cj + b, ck + c)
                verts[loc] = node2(box, 4 * I + loc[0], 4 * J + loc[1], 4 * K + loc[2])
        want = [verts[(a, b, c)] for c in range(5) for b in range(5) for a in range(5)]
        assert list(m[M]) == want
    assert int(mult.sum()) == 125 * box.n_patches
    idx = np.stack(np.meshgrid(*[np.arange(N[a]) for a in range(3)], indexing="ij"), -1).reshape(-1, 3)
    closed = np.ones(len(idx), dtype=int)
    for a in range(3):
        per = (box.periodic_mask >> a) & 1
        i = idx[:, a]
        shared = (i % 4 == 0) & (per | ((i > 0) & (i < N[a] - 1)))
        closed *= np.where(shared, 2, 1)
    nodes = idx[:, 0] + N[0] * (idx[:, 1] + N[1] * idx[:, 2])
    assert np.array_equal(mult[nodes], closed)


@pytest.mark.parametrize("name", list(BOXES))
def test_levels_one_is_the_single_level_patch(orc, name):
    box = BOXES[name]
    rng = np.random.default_rng(1)
    m1, mu1 = orc.dofmap_levels(box, 1)
    m0, mu0 = orc.dofmap(box)
    assert np.array_equal(m1, m0) and np.array_equal(mu1, mu0)
    x = rng.standard_normal((4, box.n_fine))
    r = rng.standard_normal((4, box.n_fine))
    assert np.array_equal(orc.gather_levels(box, 1, x, r), orc.gather(box, x, r))
    Y = rng.standard_normal((box.n_patches, 81))
    assert np.array_equal(orc.scatter_levels(box, 1, Y), orc.scatter(box, Y))


def interp_1d(nc, per):
    """Two-level 1-D Q1 interpolation (coarse nodes -> 4x finer nodes): fine
    node 4I + d takes weight 1 - |d|/4 from coarse node I (textbook linear
    interpolation), built directly."""
    nf = 4 * nc if per else 4 * nc + 1
    ncn = nc if per else nc + 1
    A = sp.lil_matrix((nf, ncn))
    for i in range(nf):
        I0, d = divmod(i, 4)
        A[i, I0 % ncn] += 1.0 - d / 4.0
        if d:
            A[i, (I0 + 1) % ncn] += d / 4.0
    return A.tocsr()


@pytest.mark.parametrize("name", list(BOXES))
def test_prolong_levels_is_kronecker_interpolation(orc, name):
    box = BOXES[name]
    P1 = [interp_1d(box.n[a], (box.periodic_mask >> a) & 1) for a in range(3)]
    P = sp.kron(P1[2], sp.kron(P1[1], P1[0])).tocsr()
    xc = np.random.default_rng(2).standard_normal((4, box.n_coarse))
    got = orc.prolong_levels(box, 2, xc)
    want = np.stack([P @ xc[f] for f in range(4)])
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))
    # adjointness: <R b, x> = <b, P x>
    bf = np.random.default_rng(3).standard_normal((4, P.shape[0]))
    R = orc.restrict_levels(box, 2, bf)
    assert np.allclose(R, np.stack([P.T @ bf[f] for f in range(4)]), rtol=1e-13, atol=1e-13)
    lhs = float(np.sum(R * xc))
    rhs = float(np.sum(bf * got))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_prolong_levels_reproduces_trilinear_fields(orc):
    box = BOXES["channel"]
    pc = syn.node_coords(box, fine=False)
    g = lambda p: 0.3 + 1.1 * p[0] - 0.7 * p[1] + 0.4 * p[2] + 2.0 * p[0] * p[1] * p[2] - 0.5 * p[1] * p[2]
    xc = np.stack([g(pc)] * 4)
    box4 = syn.BoxSpec(tuple(4 * n for n in box.n), box.len, box.periodic_mask, box.dirichlet_mask)
    pf = syn.node_coords(box4, fine=False)  # coarse lattice of a 4n box = the J = 2 lattice
    got = orc.prolong_levels(box, 2, xc)
    assert np.max(np.abs(got[0] - g(pf))) <= 1e-13
    assert np.all(orc.prolong_levels(box, 2, np.full((4, box.n_coarse), 2.5)) == 2.5)


@pytest.mark.parametrize("name", list(BOXES))
def test_gather_scatter_levels_consistency(orc, name):
    """L(Q(x)) = x on non-Dirichlet nodes (P:648-655 consistency of the
    averaging), conservation sum m d = sum Y, geometry columns = coarse cell
    sizes, and the standardisation is (X - shift) * inv_scale."""
    box = BOXES[name]
    box2 = orc.level_box(box, 2)
    nf = orc.fine_nodes(box2)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((4, nf))
    r = rng.standard_normal((4, nf))
    X = orc.gather_levels(box, 2, x, r)
    assert X.shape == (box.n_patches, 753)
    for a in range(3):
        assert np.all(X[:, 750 + a] == box.len[a] / box.n[a])
    d = orc.scatter_levels(box, 2, X[:, :375])
    dirf = orc.dirichlet_flags(box2).astype(bool)
    assert np.array_equal(d[:, dirf], np.zeros((3, int(dirf.sum()))))
    assert np.max(np.abs(d[:, ~dirf] - x[:3, ~dirf])) <= 4e-16 * np.max(np.abs(x))
    Y = rng.standard_normal((box.n_patches, 375))
    d = orc.scatter_levels(box, 2, Y)
    m, mult = orc.dofmap_levels(box, 2)
    for c in range(3):
        contrib = np.zeros(nf)
        np.add.at(contrib, m.ravel(), Y[:, 125 * c:125 * (c + 1)].ravel())
        assert np.allclose(d[c, ~dirf] * mult[~dirf], contrib[~dirf], rtol=1e-13, atol=1e-13)
    sh = rng.standard_normal(753)
    inv = rng.uniform(0.5, 2.0, 753)
    Xs = orc.gather_levels(box, 2, x, r, sh, inv)
    assert np.allclose(Xs, (X - sh) * inv, rtol=1e-15, atol=1e-15)


def test_lps_vanishes_on_two_level_prolongation(orc):
    """A field prolongated twice is Q1 on the coarse mesh, so on every patch
    of the next-coarser level (the LPS projection's patches) it equals its
    own interpolant: the LPS terms vanish, and the residual equals the one
    with the stabilisation switched off."""
    box = BOXES["channel"]
    box2 = orc.level_box(box, 2)
    xc = np.random.default_rng(5).standard_normal((4, box.n_coarse))
    xt = orc.prolong_levels(box, 2, xc)
    vp = xt[:3] + 0.1
    on = syn.NSParams(0.05, 0.02, 0.5, 0.8)
    off = syn.NSParams(0.05, 0.02, 0.0, 0.0)
    a, b = orc.residual(box2, on, xt, vp), orc.residual(box2, off, xt, vp)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_correction_step_levels_zero_network(orc):
    """With a zero output layer the J = 2 step makes no correction: d = 0 and
    b^L = R^2 Rhs(P^2 x^L) on the J = 2 lattice."""
    box = BOXES["channel"]
    box2 = orc.level_box(box, 2)
    ns = syn.NSParams(1e-3, 0.005)
    rng = np.random.default_rng(6)
    xc = rng.standard_normal((4, box.n_coarse))
    vp = rng.standard_normal((3, orc.fine_nodes(box2)))
    params = syn.mlp_params(753, 32, 375, seed=0)
    params[4] = np.zeros_like(params[4])
    out = orc.correction_step(box, ns, params, xc, vp, levels=2)
    assert np.all(out["d"] == 0.0)
    xt = orc.prolong_levels(box, 2, xc)
    want = orc.restrict_levels(box, 2, orc.rhs(box2, ns, xt[:3]))
    assert np.allclose(out["bc"], want, rtol=1e-14, atol=1e-14)
