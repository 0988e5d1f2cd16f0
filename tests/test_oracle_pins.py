"""Pins of the FP64 oracle against what the mathematics and the paper fix.

Each test checks the oracle against something other than itself: closed
forms, brute force over the mesh, textbook 1-D element matrices combined with
scipy.sparse.kron, invariants (nestedness, adjointness, consistency of the
patch averaging), library routines (numpy matmul, torch AdamW) and central
finite differences.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import dnnmg_synth as syn


def periodic_box(n=(4, 4, 4), L=(1.0, 1.0, 1.0)):
    return syn.BoxSpec(tuple(n), tuple(L), 7, 0)


def open_box(n=(3, 2, 2), L=(1.3, 0.7, 0.9), dirichlet=0):
    return syn.BoxSpec(tuple(n), tuple(L), 0, dirichlet)


def ns(nu=1e-3, dt=0.01, a0=0.02, d0=0.1):
    return syn.NSParams(nu, dt, a0, d0)


# ------------------------------------------------------------ 1-D textbook --

def mat1d(N, h, periodic, kind):
    """Assembled 1-D Q1 matrices on N nodes: mass h/6[1 4 1], stiffness [-1 2 -1]/h,
    C[i, j] = int phi_j' phi_i = [-1/2 0 1/2]."""
    ncell = N if periodic else N - 1
    A = np.zeros((N, N))
    if kind == "M":
        loc = h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    elif kind == "K":
        loc = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    elif kind == "C":  # row = test function, column = differentiated trial function
        loc = np.array([[-0.5, 0.5], [-0.5, 0.5]])
    for c in range(ncell):
        idx = [c, (c + 1) % N]
        for a in range(2):
            for b in range(2):
                A[idx[a], idx[b]] += loc[a, b]
    return sp.csr_matrix(A)


def kron3(Ax, Ay, Az):
    # node = i + Nx (j + Ny k): x fastest -> kron(Az, kron(Ay, Ax))
    return sp.kron(Az, sp.kron(Ay, Ax)).tocsr()


def fine_mats(box):
    Nf = box.fine_shape
    h = [box.len[a] / (2 * box.n[a]) for a in range(3)]
    per = [(box.periodic_mask >> a) & 1 for a in range(3)]
    m = {k: [mat1d(Nf[a], h[a], per[a], k) for a in range(3)] for k in "MKC"}
    return m


def prolong1d(n, periodic):
    Nc = n if periodic else n + 1
    Nf = 2 * n if periodic else 2 * n + 1
    P = np.zeros((Nf, Nc))
    for i in range(Nf):
        if i % 2 == 0:
            P[i, (i // 2) % Nc] = 1.0
        else:
            P[i, ((i - 1) // 2) % Nc] += 0.5
            P[i, ((i + 1) // 2) % Nc] += 0.5
    return sp.csr_matrix(P)


# ------------------------------------------------------------- dof map -------

@pytest.mark.parametrize("box", [periodic_box((4, 4, 4)), periodic_box((2, 4, 6)),
                                 open_box((3, 2, 2)), open_box((1, 1, 1)),
                                 syn.channel_box((4, 2, 2))])
def test_dofmap_brute_force(orc, box):
    """Patch = coarse cell = union of its 2x2x2 fine cells' vertices, ordered by
    local lattice coordinates (Sec. 4.2, dof map); valence counted directly."""
    m, mult = orc.dofmap(box)
    Nf = box.fine_shape
    per = [(box.periodic_mask >> a) & 1 for a in range(3)]

    def node(i, j, k):
        c = [i, j, k]
        for a in range(3):
            if per[a]:
                c[a] %= Nf[a]
        return c[0] + Nf[0] * (c[1] + Nf[1] * c[2])

    nx, ny, nz = box.n
    for K in range(nz):
        for J in range(ny):
            for I in range(nx):
                M = I + nx * (J + ny * K)
                verts = {}
                for dc in range(8):  # the 8 fine cells of the patch
                    ci, cj, ck = 2 * I + (dc & 1), 2 * J + ((dc >> 1) & 1), 2 * K + ((dc >> 2) & 1)
                    for v in range(8):
                        a, b, c = (dc & 1) + (v & 1), ((dc >> 1) & 1) + ((v >> 1) & 1), \
                            ((dc >> 2) & 1) + ((v >> 2) & 1)
                        verts[(c, b, a)] = node(ci + (v & 1), cj + ((v >> 1) & 1), ck + ((v >> 2) & 1))
                ordered = [verts[key] for key in sorted(verts)]
                assert len(ordered) == 27
                assert list(m[M]) == ordered
    # closed-form valence: product over axes of 2 at shared even indices
    idx = syn.lattice_index(box, True)
    expect = np.ones(box.n_fine, dtype=np.int64)
    for a in range(3):
        even = idx[a] % 2 == 0
        inner = per[a] | ((idx[a] > 0) & (idx[a] < 2 * box.n[a]))
        expect *= np.where(even & inner, 2, 1)
    assert np.array_equal(mult.astype(np.int64), expect)
    assert mult.sum() == 27 * box.n_patches
    assert set(np.unique(mult)).issubset({1, 2, 4, 8})


# -------------------------------------------------- prolongation / restriction

@pytest.mark.parametrize("box", [periodic_box((4, 4, 4)), open_box((3, 2, 2)), periodic_box((2, 6, 4))])
def test_prolong_kronecker(orc, box):
    """Q1 prolongation = tensor product of the 1-D [1/2, 1, 1/2] interpolation."""
    per = [(box.periodic_mask >> a) & 1 for a in range(3)]
    P = kron3(*[prolong1d(box.n[a], per[a]) for a in range(3)])
    xc = syn.random_coarse_field(box, 4, 3)
    xf = orc.prolong(box, xc)
    for c in range(4):
        np.testing.assert_allclose(xf[c], P @ xc[c], rtol=0, atol=1e-14)


def test_prolong_constants_and_trilinear(orc):
    box = open_box((3, 2, 4), (1.5, 0.5, 2.0))
    ones = np.ones((2, box.n_coarse)) * np.array([[1.25], [-3.5]])
    xf = orc.prolong(box, ones)
    assert np.array_equal(xf, np.ones((2, box.n_fine)) * np.array([[1.25], [-3.5]]))
    # a global trilinear function is reproduced at every fine node
    pc, pf = syn.node_coords(box, False), syn.node_coords(box, True)
    f = lambda p: 0.3 + 1.1 * p[0] - 0.7 * p[1] + 0.2 * p[2] + 0.5 * p[0] * p[1] \
        - 0.9 * p[1] * p[2] + 0.4 * p[0] * p[2] + 1.3 * p[0] * p[1] * p[2]
    out = orc.prolong(box, f(pc)[None])
    np.testing.assert_allclose(out[0], f(pf), rtol=0, atol=1e-14)
    # injection at coincident nodes
    idx = syn.lattice_index(box, True)
    even = np.all(idx % 2 == 0, axis=0)
    xc = syn.random_coarse_field(box, 1, 5)
    assert np.array_equal(np.sort(orc.prolong(box, xc)[0][even]), np.sort(xc[0]))


@pytest.mark.parametrize("box", [periodic_box((4, 2, 6)), open_box((3, 2, 2))])
def test_restrict_adjoint(orc, box):
    """Restriction is the transpose of prolongation: <R b, x> = <b, P x>; rows of P sum to 1."""
    b = syn.random_fine_field(box, 2, 7)
    x = syn.random_coarse_field(box, 2, 8)
    Rb = orc.restrict(box, b)
    Px = orc.prolong(box, x)
    for c in range(2):
        lhs, rhs = Rb[c] @ x[c], b[c] @ Px[c]
        assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1)
        np.testing.assert_allclose(Rb[c].sum(), b[c].sum(), rtol=1e-13)


def test_restrict_galerkin_mass(orc):
    """Nested spaces: P^T M_fine P = M_coarse (exact mass matrices via kron)."""
    box = periodic_box((4, 6, 4), (1.0, 1.5, 0.8))
    per = [1, 1, 1]
    Mf = kron3(*fine_mats(box)["M"])
    H = [box.len[a] / box.n[a] for a in range(3)]
    Mc = kron3(*[mat1d(box.n[a], H[a], 1, "M") for a in range(3)])
    x = syn.random_coarse_field(box, 1, 1)[0]
    lhs = orc.restrict(box, (Mf @ orc.prolong(box, x[None])[0])[None])[0]
    np.testing.assert_allclose(lhs, Mc @ x, rtol=1e-12, atol=1e-15)
    del per


# ------------------------------------------------------------- residual ------

def test_residual_zero_at_rest_and_mass_closed_form(orc):
    box = periodic_box((4, 4, 4))
    p = ns()
    nf = box.n_fine
    c = np.array([0.3, -1.2, 0.7])
    x = np.zeros((4, nf)); x[:3] = c[:, None]
    r = orc.residual(box, p, x, x[:3].copy())
    assert np.max(np.abs(r)) <= 1e-13
    # constant v, different constant vp: only the mass term, row sums h^3 / k
    vp = x[:3] + np.array([0.5, 0.25, -1.0])[:, None]
    r = orc.residual(box, p, x, vp)
    h3 = (1.0 / 8) ** 3
    for a in range(3):
        np.testing.assert_allclose(r[a], (vp[a] - x[a]) * h3 / p.dt, rtol=1e-12)
    assert np.max(np.abs(r[3])) <= 1e-14


@pytest.mark.parametrize("box", [periodic_box((2, 2, 2), (1.0, 0.6, 1.4)),
                                 open_box((2, 1, 2), (1.0, 0.5, 0.8))])
def test_residual_linear_parts_kronecker(orc, box):
    """Mass, stiffness, pressure-gradient and divergence parts equal the
    Kronecker products of the textbook 1-D Q1 matrices."""
    nf = box.n_fine
    m = fine_mats(box)
    Mx, My, Mz = m["M"]; Kx, Ky, Kz = m["K"]; Cx, Cy, Cz = m["C"]
    M3 = kron3(Mx, My, Mz)
    K3 = kron3(Kx, My, Mz) + kron3(Mx, Ky, Mz) + kron3(Mx, My, Kz)
    C3 = [kron3(Cx, My, Mz), kron3(Mx, Cy, Mz), kron3(Mx, My, Cz)]
    rng = np.random.default_rng(11)
    zero4 = np.zeros((4, nf))
    # pressure only (a coarse-Q1 pressure keeps the alpha-LPS term at zero)
    pc = rng.standard_normal((1, box.n_coarse))
    x = zero4.copy(); x[3] = orc.prolong(box, pc)[0]
    r = orc.residual(box, ns(), x, np.zeros((3, nf)))
    for a in range(3):  # +(p, d_a phi_i) = (C_a^T p)_i
        np.testing.assert_allclose(r[a], C3[a].T @ x[3], rtol=1e-11, atol=1e-13)
    # linear part in vp with v = 0: odd part of r(vp) = (1/k) M vp - nu/2 K vp
    vp = rng.standard_normal((3, nf))
    for nu, dt in [(0.0, 0.01), (0.3, 1e300)]:
        P = ns(nu=nu, dt=dt)
        rp = orc.residual(box, P, zero4, vp)
        rm = orc.residual(box, P, zero4, -vp)
        for a in range(3):
            odd = 0.5 * (rp[a] - rm[a])
            expect = (1.0 / dt) * (M3 @ vp[a]) - 0.5 * nu * (K3 @ vp[a])
            np.testing.assert_allclose(odd, expect, rtol=1e-11, atol=1e-12 * np.abs(expect).max())
    # divergence: -(div v, xi) with p = 0 (alpha-LPS vanishes)
    x = zero4.copy(); x[:3] = rng.standard_normal((3, nf))
    r = orc.residual(box, ns(), x, x[:3].copy())
    expect = -(C3[0] @ x[0] + C3[1] @ x[1] + C3[2] @ x[2])
    np.testing.assert_allclose(r[3], expect, rtol=1e-11, atol=1e-13)


def test_residual_convection_by_constant_field(orc):
    """With v = c + eps u (u coarse-Q1 so the LPS terms vanish), the part of the
    residual linear in eps contains -(1/2)(c . grad u_a, phi_i) = Kronecker C stencils."""
    box = periodic_box((2, 2, 2), (1.0, 0.8, 1.2))
    nf = box.n_fine
    m = fine_mats(box)
    Mx, My, Mz = m["M"]; Cx, Cy, Cz = m["C"]; Kx, Ky, Kz = m["K"]
    C3 = [kron3(Cx, My, Mz), kron3(Mx, Cy, Mz), kron3(Mx, My, Cz)]
    M3 = kron3(Mx, My, Mz)
    K3 = kron3(Kx, My, Mz) + kron3(Mx, Ky, Mz) + kron3(Mx, My, Kz)
    c = np.array([0.7, -0.4, 1.1])
    u = orc.prolong(box, syn.random_coarse_field(box, 3, 4))
    P = ns(nu=0.01, dt=0.1)
    eps = 1e-3

    def r_of(e):
        x = np.zeros((4, nf)); x[:3] = c[:, None] + e * u
        # vp = v so the mass term is zero; vp terms add the same convection again
        return orc.residual(box, P, x, x[:3].copy())

    lin = (r_of(eps) - r_of(-eps)) / (2 * eps)
    for a in range(3):
        conv = sum(c[d] * (C3[d] @ u[a]) for d in range(3))
        # two copies of -1/2 (c.grad u) (v and vp) and two of -nu/2 K u
        expect = -conv - P.nu * (K3 @ u[a])
        np.testing.assert_allclose(lin[a], expect, rtol=1e-8, atol=1e-9 * np.abs(expect).max())
    del M3


def test_residual_convection_energy_identity(orc):
    """sum_i v_a(i) [(v.grad v_a), phi_i] = -1/2 int (div v)|v|^2 on a periodic box,
    with the right side integrated independently by 3-point Gauss."""
    box = periodic_box((2, 2, 2), (1.0, 1.0, 1.0))
    nf = box.n_fine
    rng = np.random.default_rng(3)
    v = rng.standard_normal((3, nf))
    P = ns(nu=0.0, dt=1e300, a0=0.0, d0=0.0)
    x = np.zeros((4, nf)); x[:3] = v
    # r = -1/2 N(vp) - 1/2 N(v) with vp = v -> -N(v)
    r = orc.residual(box, P, x, v.copy())
    lhs = -np.sum(v * r[:3])
    # independent integral of -1/2 (div v)|v|^2 over the trilinear interpolant
    Nf = box.fine_shape
    h = [box.len[a] / Nf[a] for a in range(3)]
    V = v.reshape(3, Nf[2], Nf[1], Nf[0])
    g, w = np.polynomial.legendre.leggauss(3)
    g = 0.5 * (g + 1); w = 0.5 * w
    total = 0.0
    for ck in range(Nf[2]):
        for cj in range(Nf[1]):
            for ci in range(Nf[0]):
                vals = np.zeros((3, 2, 2, 2))
                for c_ in range(2):
                    for b_ in range(2):
                        for a_ in range(2):
                            vals[:, c_, b_, a_] = V[:, (ck + c_) % Nf[2], (cj + b_) % Nf[1], (ci + a_) % Nf[0]]
                for qz, wz in zip(g, w):
                    for qy, wy in zip(g, w):
                        for qx, wx in zip(g, w):
                            lz = np.array([1 - qz, qz]); ly = np.array([1 - qy, qy]); lx = np.array([1 - qx, qx])
                            d = np.array([-1.0, 1.0])
                            val = np.einsum("zcba,c,b,a->z", vals, lz, ly, lx)
                            dx = np.einsum("zcba,c,b,a->z", vals, lz, ly, d) / h[0]
                            dy = np.einsum("zcba,c,b,a->z", vals, lz, d, lx) / h[1]
                            dz = np.einsum("zcba,c,b,a->z", vals, d, ly, lx) / h[2]
                            div = dx[0] + dy[1] + dz[2]
                            total += wx * wy * wz * h[0] * h[1] * h[2] * (-0.5 * div * val.dot(val))
    assert abs(lhs - total) <= 1e-11 * max(1.0, abs(total))


def test_residual_galerkin_nested_levels(orc):
    """Nested Q1 spaces with exact quadrature: R(r_fine(P x, P vp)) = r_coarse(x, vp)
    for the Galerkin terms (LPS switched off, periodic box, no Dirichlet rows)."""
    fine_box = periodic_box((4, 2, 4), (1.0, 0.6, 1.2))
    coarse_as_fine = periodic_box((2, 1, 2), (1.0, 0.6, 1.2))
    P = ns(nu=0.05, dt=0.02, a0=0.0, d0=0.0)
    rng = np.random.default_rng(5)
    nc = fine_box.n_coarse
    x = rng.standard_normal((4, nc)); vp = rng.standard_normal((3, nc))
    fm = rng.standard_normal((3, nc))
    rf = orc.residual(fine_box, P, orc.prolong(fine_box, x), orc.prolong(fine_box, vp),
                      orc.prolong(fine_box, fm))
    lhs = orc.restrict(fine_box, rf)
    rc = orc.residual(coarse_as_fine, P, x, vp, fm)
    np.testing.assert_allclose(lhs, rc, rtol=1e-10, atol=1e-12 * np.abs(rc).max())
    # same for the right-hand side of the next step
    bf = orc.rhs(fine_box, P, orc.prolong(fine_box, vp), orc.prolong(fine_box, fm))
    bc = orc.rhs(coarse_as_fine, P, vp, fm)
    np.testing.assert_allclose(orc.restrict(fine_box, bf), bc, rtol=1e-10, atol=1e-12 * np.abs(bc).max())


def test_residual_equals_rhs_minus_operator(orc):
    """r(x; vp) = Rhs(vp) - A(x): the residual at x = (vp, p) with the same field
    reduces to the operator difference; here check additivity in vp."""
    box = syn.channel_box((2, 1, 1))
    P = ns()
    rng = np.random.default_rng(9)
    nf = box.n_fine
    x = rng.standard_normal((4, nf)); vp = rng.standard_normal((3, nf)); f = rng.standard_normal((3, nf))
    r = orc.residual(box, P, x, vp, f)
    r0 = orc.residual(box, P, x, np.zeros((3, nf)))
    b = orc.rhs(box, P, vp, f)
    np.testing.assert_allclose(r, r0 + b, rtol=1e-11, atol=1e-12 * np.abs(r).max())


def test_lps_vanishes_on_prolongated_fields(orc):
    """The two-level LPS terms vanish at x = P x^L (x is in the coarse space):
    switching them on or off changes nothing there."""
    box = periodic_box((4, 2, 2), (1.0, 0.5, 0.5))
    rng = np.random.default_rng(2)
    x = orc.prolong(box, rng.standard_normal((4, box.n_coarse)))
    vp = rng.standard_normal((3, box.n_fine))
    r_on = orc.residual(box, ns(), x, vp)
    r_off = orc.residual(box, ns(a0=0.0, d0=0.0), x, vp)
    np.testing.assert_allclose(r_on, r_off, rtol=0, atol=1e-13 * np.abs(r_off).max())
    # but not on a general fine field
    x2 = x + 0.1 * rng.standard_normal(x.shape)
    r_on = orc.residual(box, ns(), x2, vp)
    r_off = orc.residual(box, ns(a0=0.0, d0=0.0), x2, vp)
    assert np.max(np.abs(r_on - r_off)) > 1e-8


def test_lps_pressure_term_psd(orc):
    """alpha-term is a symmetric positive semidefinite form in p (v = 0)."""
    box = periodic_box((2, 2, 2))
    rng = np.random.default_rng(4)
    nf = box.n_fine
    for _ in range(3):
        x = np.zeros((4, nf)); x[3] = rng.standard_normal(nf)
        r = orc.residual(box, ns(a0=0.5), x, np.zeros((3, nf)))
        # r_p = -alpha (grad(p - pi p), grad(xi - pi xi)) -> p . r_p <= 0
        assert x[3] @ r[3] <= 1e-14


def test_residual_translation_equivariance(orc):
    """Shifting all fields by one coarse cell on a periodic box shifts the residual."""
    box = periodic_box((4, 2, 2), (1.0, 0.5, 0.5))
    rng = np.random.default_rng(6)
    nf = box.n_fine
    Nf = box.fine_shape
    x = rng.standard_normal((4, nf)); vp = rng.standard_normal((3, nf))

    def shift(a):
        return np.roll(a.reshape(a.shape[0], Nf[2], Nf[1], Nf[0]), 2, axis=3).reshape(a.shape[0], nf)

    r = orc.residual(box, ns(), x, vp)
    rs = orc.residual(box, ns(), shift(x), shift(vp))
    np.testing.assert_allclose(rs, shift(r), rtol=1e-12, atol=1e-14 * np.abs(r).max())


def test_dirichlet_rows_zero(orc):
    box = syn.channel_box((2, 1, 1))
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, box.n_fine)); vp = rng.standard_normal((3, box.n_fine))
    r = orc.residual(box, ns(), x, vp)
    dmask = syn.boundary_mask(box, True)
    assert np.array_equal(orc.dirichlet_flags(box).astype(bool), dmask)
    assert np.all(r[:3, dmask] == 0.0)
    assert np.all(np.abs(r[:3, ~dmask]) > 0)
    b = orc.rhs(box, ns(), vp)
    assert np.all(b[:3, dmask] == 0.0) and np.all(b[3] == 0.0)


# ------------------------------------------------------- gather / scatter ---

@pytest.mark.parametrize("box", [periodic_box((4, 2, 2)), syn.channel_box((3, 2, 2))])
def test_scatter_of_gather_is_identity(orc, box):
    """L(Q(x)) = x on every free node: averaging identical copies (eq. defL)."""
    rng = np.random.default_rng(8)
    x = np.zeros((4, box.n_fine)); x[:3] = rng.standard_normal((3, box.n_fine))
    r = rng.standard_normal((4, box.n_fine))
    X = orc.gather(box, x, r)
    d = orc.scatter(box, X[:, :81])
    free = ~syn.boundary_mask(box, True)
    np.testing.assert_allclose(d[:, free], x[:3, free], rtol=0, atol=4e-16 * 8)
    assert np.all(d[:, ~free] == 0.0)
    # residual block and cell sizes
    X2 = orc.gather(box, r, x)
    np.testing.assert_allclose(orc.scatter(box, X2[:, 81:162])[:, free], x[:3, free], atol=1e-15 * 8)
    H = [box.len[a] / box.n[a] for a in range(3)]
    assert np.allclose(X[:, 162:], np.array(H)[None, :], rtol=0, atol=0)


def test_scatter_conservation_and_permutation(orc):
    box = periodic_box((4, 2, 2))
    rng = np.random.default_rng(10)
    Y = rng.standard_normal((box.n_patches, 81))
    d = orc.scatter(box, Y)
    _, mult = orc.dofmap(box)
    np.testing.assert_allclose((d * mult[None, :]).sum(axis=1),
                               Y.reshape(-1, 3, 27).sum(axis=(0, 2)), rtol=1e-12)


def test_gather_standardisation(orc):
    box = periodic_box((2, 2, 2))
    rng = np.random.default_rng(12)
    x = rng.standard_normal((4, box.n_fine)); r = rng.standard_normal((4, box.n_fine))
    sh = rng.standard_normal(165); sc = rng.uniform(0.5, 2.0, 165)
    np.testing.assert_allclose(orc.gather(box, x, r, sh, sc), (orc.gather(box, x, r) - sh) * sc, rtol=1e-15)


# ------------------------------------------------------------ network -------

def test_mlp_forward_matches_matmul(orc):
    rng = np.random.default_rng(0)
    W1, b1, W2, b2, W3, b3 = syn.mlp_params(165, 16, 81, seed=1, bias_scale=0.1)
    X = rng.standard_normal((9, 165))
    Y = orc.mlp_forward(X, W1, b1, W2, b2, W3, b3)
    ref = np.tanh(np.tanh(X @ W1 + b1) @ W2 + b2) @ W3 + b3
    np.testing.assert_allclose(Y, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dims", [(7, 5, 3), (165, 8, 81)])
def test_mlp_backward_finite_differences(orc, dims):
    nin, H, nout = dims
    rng = np.random.default_rng(1)
    params = syn.mlp_params(nin, H, nout, seed=2, bias_scale=0.2)
    X = rng.standard_normal((6, nin)); T = rng.standard_normal((6, nout))

    def loss(ps):
        return orc.mse(orc.mlp_forward(X, *ps), T)[0]

    Y, A1, A2 = orc.mlp_forward(X, *params, want_hidden=True)
    _, dY = orc.mse(Y, T)
    grads = orc.mlp_backward(X, params[2], params[4], A1, A2, dY)
    h = 1e-6
    for pi, g in enumerate(grads):
        flat = params[pi].ravel()
        sel = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for s in sel:
            pp = [p.copy() for p in params]; pm = [p.copy() for p in params]
            pp[pi].ravel()[s] += h; pm[pi].ravel()[s] -= h
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(fd - g.ravel()[s]) <= 1e-6 * max(1.0, abs(fd)), (pi, s, fd, g.ravel()[s])


def test_adamw_matches_torch(orc):
    import torch

    rng = np.random.default_rng(3)
    theta0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(10)]
    lr, b1, b2, eps, wd = 1e-3, 0.9, 0.999, 1e-8, 1e-5
    th = theta0.copy(); m = np.zeros(50); v = np.zeros(50)
    for t, g in enumerate(grads, start=1):
        orc.adamw(th, m, v, g, lr, b1, b2, eps, wd, t)
    p = torch.nn.Parameter(torch.tensor(theta0, dtype=torch.float64))
    opt = torch.optim.AdamW([p], lr=lr, betas=(b1, b2), eps=eps, weight_decay=wd)
    for g in grads:
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_rounding_formats_match_torch(orc):
    import torch

    rng = np.random.default_rng(4)
    # float32-representable inputs (the GPU path rounds from FP32)
    x = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 3, 2000),
                        [0.0, 1.0, -1.0, 448.0, -448.0, 2.0 ** -9, 3 * 2.0 ** -10]])
    x = x.astype(np.float32).astype(np.float64)
    bf = torch.tensor(x, dtype=torch.float64).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(orc.round_bf16(x), bf)
    inr = np.abs(x) <= 448.0
    f8 = torch.tensor(x[inr], dtype=torch.float64).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(orc.round_e4m3(x[inr]), f8)
    assert orc.round_e4m3(np.array([500.0, -1e6])).tolist() == [448.0, -448.0]


def test_lps_convection_term_sign(orc):
    """Testing the delta-term with the velocity itself gives
    sum_T delta_T int |v.grad v - pi v.grad pi v|^2 >= 0, so switching the term
    on lowers v . r; it also scales linearly in delta0."""
    box = periodic_box((2, 2, 2))
    rng = np.random.default_rng(14)
    nf = box.n_fine
    for _ in range(3):
        x = np.zeros((4, nf)); x[:3] = rng.standard_normal((3, nf))
        vp = rng.standard_normal((3, nf))
        r_off = orc.residual(box, ns(a0=0.0, d0=0.0), x, vp)
        r_on = orc.residual(box, ns(a0=0.0, d0=0.1), x, vp)
        r_on2 = orc.residual(box, ns(a0=0.0, d0=0.2), x, vp)
        e = np.sum(x[:3] * (r_on - r_off)[:3])
        assert e < 0.0
        np.testing.assert_allclose(r_on2 - r_off, 2 * (r_on - r_off), rtol=1e-9,
                                   atol=1e-12 * np.abs(r_on - r_off).max())


# ------------------------------------------- plain fine correction (Vanka) --

def fd_jacobian(orc, box, P, x0, vp, eps=1e-6):
    """-dr/dx by central differences of the oracle residual."""
    nf = box.n_fine
    J = np.zeros((4 * nf, 4 * nf))
    for c in range(4 * nf):
        e = np.zeros(4 * nf); e[c] = eps
        rp = orc.residual(box, P, (x0.ravel() + e).reshape(4, nf), vp)
        rm = orc.residual(box, P, (x0.ravel() - e).reshape(4, nf), vp)
        J[:, c] = -(rp - rm).ravel() / (2 * eps)
    return J


def to_local(box, A_global, orc):
    """Reorder a global [field][node] matrix of a one-patch box to the local
    [field][iota] ordering (the dof map of the single patch)."""
    m, _ = orc.dofmap(box)
    nf = box.n_fine
    idx = np.concatenate([f * nf + m[0] for f in range(4)])
    return A_global[np.ix_(idx, idx)]


def test_vanka_matrix_is_jacobian_at_rest(orc):
    """On a box that is one patch, the local matrix at w = 0 equals the exact
    Jacobian of the Crank-Nicolson operator (finite differences of the
    residual): mass, viscosity, pressure gradient, divergence and the
    pressure LPS term."""
    box = open_box((1, 1, 1), (0.7, 0.5, 0.9))
    P = ns(nu=0.03, dt=0.02, a0=0.3)
    nf = box.n_fine
    J = to_local(box, fd_jacobian(orc, box, P, np.zeros((4, nf)), np.zeros((3, nf))), orc)
    A = orc.vanka_matrix(box, P, np.zeros((3, nf)), 0)
    np.testing.assert_allclose(A, J, rtol=1e-6, atol=1e-9 * np.abs(J).max())


def test_vanka_matrix_rows_are_global_rows(orc):
    """On a periodic box, with the LPS terms off, the local matrix at w = 0 is
    the exact Jacobian restricted to the patch's rows and columns (it
    includes the neighbouring cells' contributions to shared rows)."""
    box = periodic_box((2, 2, 2), (1.0, 0.8, 1.2))
    P = ns(nu=0.03, dt=0.02, a0=0.0, d0=0.0)
    nf = box.n_fine
    Jg = fd_jacobian(orc, box, P, np.zeros((4, nf)), np.zeros((3, nf)))
    m, _ = orc.dofmap(box)
    for M in (0, 5):
        idx = np.concatenate([f * nf + m[M] for f in range(4)])
        A = orc.vanka_matrix(box, P, np.zeros((3, nf)), M)
        np.testing.assert_allclose(A, Jg[np.ix_(idx, idx)], rtol=1e-6, atol=1e-9 * np.abs(Jg).max())


def test_vanka_matrix_convection_constant_field(orc):
    """With a constant velocity c the Picard convection block is
    1/2 sum_d c_d C_d (Kronecker products of textbook 1-D matrices)."""
    box = open_box((1, 1, 1), (0.7, 0.5, 0.9))
    P = ns(nu=0.03, dt=0.02, a0=0.0)
    nf = box.n_fine
    c = np.array([0.4, -0.9, 0.3])
    A0 = orc.vanka_matrix(box, P, np.zeros((3, nf)), 0)
    Ac = orc.vanka_matrix(box, P, np.tile(c[:, None], (1, nf)), 0)
    m = fine_mats(box)
    Mx, My, Mz = m["M"]; Cx, Cy, Cz = m["C"]
    C3 = [kron3(Cx, My, Mz), kron3(Mx, Cy, Mz), kron3(Mx, My, Cz)]
    conv = 0.5 * sum(c[d] * C3[d].toarray() for d in range(3))
    mp, _ = orc.dofmap(box)
    conv = conv[np.ix_(mp[0], mp[0])]
    for a in range(3):
        blk = slice(27 * a, 27 * a + 27)
        np.testing.assert_allclose((Ac - A0)[blk, blk], conv, rtol=1e-10, atol=1e-14)
    # only the velocity-velocity blocks change
    Ac[:81, :81] = A0[:81, :81]
    np.testing.assert_array_equal(Ac, A0)


def test_vanka_matrix_dirichlet_identity(orc):
    box = syn.channel_box((1, 1, 1))
    nf = box.n_fine
    A = orc.vanka_matrix(box, ns(), np.random.default_rng(0).standard_normal((3, nf)), 0)
    dmask = syn.boundary_mask(box, True)
    mp, _ = orc.dofmap(box)
    for t in range(27):
        if dmask[mp[0][t]]:
            for a in range(3):
                r = 27 * a + t
                e = np.zeros(108); e[r] = 1.0
                assert np.array_equal(A[r], e) and np.array_equal(A[:, r], e)


def test_dense_solve_matches_numpy(orc):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((108, 108)); b = rng.standard_normal(108)
    np.testing.assert_allclose(orc.dense_solve(A, b), np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("coupled", [True, False])
def test_vanka_sweep_composition(orc, coupled):
    """A sweep adds the L-average of the local solutions, checked against
    numpy.linalg.solve on every patch (full system, or the velocity block per
    component with the pressure held)."""
    box = syn.BoxSpec((2, 2, 2), (1.0, 1.0, 1.0), 7, 0)
    P = syn.cfg1().ns
    rng = np.random.default_rng(2)
    nf = box.n_fine
    modes = syn.fourier_modes(rng)
    vp = syn.fourier_velocity(modes, syn.node_coords(box, True), box.len)
    x = np.zeros((4, nf)); x[:3] = vp + 0.05 * rng.standard_normal((3, nf))
    x[3] = 0.1 * rng.standard_normal(nf)
    out = orc.vanka_sweep(box, P, x, vp, omega=0.7, coupled=coupled)
    r = orc.residual(box, P, x, vp)
    m, mult = orc.dofmap(box)
    d = np.zeros((4, nf))
    for M in range(box.n_patches):
        A = orc.vanka_matrix(box, P, x[:3], M)
        rhs = np.concatenate([r[f][m[M]] for f in range(4)])
        if coupled:
            dl = np.linalg.solve(A, rhs)
        else:
            dl = np.concatenate([np.linalg.solve(A[:27, :27], rhs[27 * a: 27 * a + 27]) for a in range(3)]
                                + [np.zeros(27)])
        for f in range(4):
            np.add.at(d[f], m[M], dl[27 * f: 27 * f + 27])
    np.testing.assert_allclose(out, x + 0.7 * d / mult[None, :], rtol=1e-9, atol=1e-12)
    if not coupled:
        assert np.array_equal(out[3], x[3])


@pytest.mark.parametrize("box", [syn.channel_box((4, 2, 2)), syn.cfg1().box])
def test_vanka_velocity_sweeps_converge(orc, box):
    """The pressure-held sweeps drive the momentum residual down geometrically
    (rough prolongated field, factor >= 3 per sweep), leaving the pressure."""
    P = syn.NSParams(1e-3, 0.005)
    rng = np.random.default_rng(3)
    x = orc.prolong(box, rng.standard_normal((4, box.n_coarse)))
    vp = x[:3] + 0.2 * rng.standard_normal((3, box.n_fine))
    dm = syn.boundary_mask(box, True)
    vp[:, dm] = x[:3, dm]
    norms = []
    for _ in range(4):
        norms.append(np.linalg.norm(orc.residual(box, P, x, vp)[:3]))
        x = orc.vanka_sweep(box, P, x, vp, omega=1.0, coupled=False)
    norms.append(np.linalg.norm(orc.residual(box, P, x, vp)[:3]))
    for a, b in zip(norms, norms[1:]):
        assert b < a / 3.0, norms


def test_scatter_independent_of_summation_order(orc):
    """Extension L (eq. defL) summed in a random order of the (patch, local
    node) pairs with numpy, from the brute-force dof lists: the oracle's
    fixed-order sums agree to roundoff; relabelling the patches by a
    periodic translation of one coarse cell shifts d by two fine nodes."""
    box = periodic_box((4, 2, 2), (1.0, 0.5, 0.5))
    rng = np.random.default_rng(31)
    Y = rng.standard_normal((box.n_patches, 81))
    d = orc.scatter(box, Y)
    Nf = box.fine_shape
    acc = np.zeros((3, box.n_fine)); cnt = np.zeros(box.n_fine)
    pairs = [(M, a, b, c) for M in range(box.n_patches) for c in range(3) for b in range(3) for a in range(3)]
    for t in rng.permutation(len(pairs)):
        M, a, b, c = pairs[t]
        I = M % box.n[0]; J = (M // box.n[0]) % box.n[1]; K = M // (box.n[0] * box.n[1])
        g = ((2 * I + a) % Nf[0]) + Nf[0] * (((2 * J + b) % Nf[1]) + Nf[1] * ((2 * K + c) % Nf[2]))
        for comp in range(3):
            acc[comp, g] += Y[M, 27 * comp + a + 3 * b + 9 * c]
        cnt[g] += 1
    np.testing.assert_allclose(d, acc / cnt[None, :], rtol=1e-14, atol=1e-15)
    # translation: patch (I, J, K) -> (I+1, J, K)
    Yr = Y.reshape(box.n[2], box.n[1], box.n[0], 81)
    Ys = np.roll(Yr, 1, axis=2).reshape(-1, 81)
    ds = orc.scatter(box, Ys)
    shift = lambda a: np.roll(a.reshape(3, Nf[2], Nf[1], Nf[0]), 2, axis=3).reshape(3, -1)
    np.testing.assert_allclose(ds, shift(d), rtol=1e-14, atol=1e-15)


def test_mse_matches_torch(orc):
    """Training loss (1/n) sum_M ||Y_M - T_M||^2 and its gradient against
    torch's mse_loss and autograd."""
    import torch

    rng = np.random.default_rng(32)
    Y = rng.standard_normal((37, 81)); T = rng.standard_normal((37, 81))
    loss, dY = orc.mse(Y, T)
    y = torch.tensor(Y, dtype=torch.float64, requires_grad=True)
    ref = torch.nn.functional.mse_loss(y, torch.tensor(T, dtype=torch.float64), reduction="sum") / Y.shape[0]
    ref.backward()
    assert abs(loss - ref.item()) <= 1e-13 * ref.item()
    np.testing.assert_allclose(dY, y.grad.numpy(), rtol=1e-13, atol=1e-16)


def test_mlp_rows_on_threads_equal_one_call(orc):
    """The network evaluated over row ranges on host threads gives the one-call
    result bit for bit (each row's arithmetic is the same)."""
    import dnnmg_synth as syn

    params = syn.mlp_params(165, 64, 81, seed=3, bias_scale=0.1)
    X = np.random.default_rng(4).standard_normal((1001, 165))
    a = orc.mlp_forward(X, *params)
    b = orc.mlp_forward_rows(X, params, threads=7)
    assert np.array_equal(a, b)
