"""Pins of the Q2/Q2 oracle (Sec. 2.2 eq. (disc:ns) with equal-order Q2
elements and pi_h: Q2 -> Q1; Sec. 2.3 eq. (4cranknicholson3), (stabparams);
the transfer of Algorithm 1 between the Q2 spaces of two levels).

Each pin checks the oracle against something it does not compute itself:
  * on axis-parallel meshes the Galerkin terms are Kronecker products of the
    1-D quadratic element matrices, integrated exactly here with numpy
    polynomials;
  * on affine meshes quadratic and linear fields are reproduced, so the
    stiffness, pressure, divergence and convection terms reduce to closed
    forms times the row sums of the mass matrix (det A times the lattice's);
  * on a curved isoparametric mesh (a global quadratic map) the volume and
    the gradients of linear fields are exact;
  * rigid motions leave the scalar rows unchanged and rotate the momentum
    rows;
  * both LPS terms vanish on element-wise Q1 fields, and their magnitudes
    are element sums of (I - Pi_T)^T K_T (I - Pi_T) with Pi_T the Kronecker
    product of the 1-D interpolation onto the element's end points;
  * the prolongation reproduces global quadratics, the restriction is its
    transpose, and R A_fine(P x) = A_coarse(x) for the linear terms;
  * altered copies of the oracle (h_T, each term of eq. (stabparams), either
    LPS term scaled) fail at least one pin.
"""
import contextlib
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.sparse as sp
from numpy.polynomial import Polynomial as Poly

import dnnmg_synth as syn
from test_oracle_pins import kron3


@pytest.fixture(scope="module")
def q2():
    from oracle import q2 as mod

    mod.lib()
    return mod


def box_of(n, lens=(1.0, 1.0, 1.0), dmask=0):
    return syn.BoxSpec(tuple(n), tuple(lens), 0, dmask)


def lattice(box):
    """Node positions of the undistorted box: element size len / n, so the
    node spacing is half of it."""
    return syn.node_coords(box, fine=True)


def ns_of(nu, dt, a0=0.0, d0=0.0):
    return syn.NSParams(nu, dt, a0, d0)


# ----------------------------------------------------- 1-D element matrices --

def q2_basis(H):
    ts = [0.0, 0.5 * H, H]
    out = []
    for i in range(3):
        p = Poly([1.0])
        for j in range(3):
            if j != i:
                p = p * Poly([-ts[j], 1.0]) / (ts[i] - ts[j])
        out.append(p)
    return out


def elem1d(H):
    """Exact 1-D element matrices on [0, H]: M_ij = int phi_i phi_j,
    K_ij = int phi_i' phi_j', C_ij = int phi_i' phi_j."""
    b = q2_basis(H)

    def integ(p):
        P = p.integ()
        return P(H) - P(0.0)

    M = np.array([[integ(b[i] * b[j]) for j in range(3)] for i in range(3)])
    K = np.array([[integ(b[i].deriv() * b[j].deriv()) for j in range(3)] for i in range(3)])
    C = np.array([[integ(b[i].deriv() * b[j]) for j in range(3)] for i in range(3)])
    return dict(M=M, K=K, C=C)


def glob1d(n, H):
    e = elem1d(H)
    out = {}
    for k, E in e.items():
        G = np.zeros((2 * n + 1, 2 * n + 1))
        for el in range(n):
            s = slice(2 * el, 2 * el + 3)
            G[s, s] += E
        out[k] = sp.csr_matrix(G)
    return out


def mats3(box):
    m = [glob1d(box.n[a], box.len[a] / box.n[a]) for a in range(3)]
    M = kron3(m[0]["M"], m[1]["M"], m[2]["M"])
    K = (kron3(m[0]["K"], m[1]["M"], m[2]["M"]) + kron3(m[0]["M"], m[1]["K"], m[2]["M"])
         + kron3(m[0]["M"], m[1]["M"], m[2]["K"]))
    # B[a][i, j] = int phi_j d_a phi_i ; D[a][i, j] = int d_a phi_j phi_i
    Ms = [m[a]["M"] for a in range(3)]
    B, D = [], []
    for a in range(3):
        f = list(Ms)
        f[a] = m[a]["C"]
        B.append(kron3(*f))
        f[a] = m[a]["C"].T.tocsr()
        D.append(kron3(*f))
    return M, K, B, D


def odd_even(q2, box, ns, X, x):
    Ap = q2.apply(box, ns, X, x)
    Am = q2.apply(box, ns, X, -x)
    return 0.5 * (Ap - Am), 0.5 * (Ap + Am)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------- basis ----

def test_q2_mesh_counts(q2):
    box = box_of((3, 2, 4))
    assert q2.fine_nodes(box) == 7 * 5 * 9
    assert q2.coarse_nodes(box) == 4 * 3 * 5
    assert q2.elements(box) == 24


# ------------------------------------------ Galerkin terms, lattice meshes --

@pytest.mark.parametrize("n,lens", [((2, 2, 2), (1.0, 0.7, 1.3)), ((3, 2, 1), (0.9, 0.5, 0.4))])
def test_q2_linear_terms_are_kronecker_products(q2, n, lens):
    """Odd part of A at alpha0 = delta0 = 0: (1/k) M v_a + nu/2 K v_a - B_a p
    in the momentum rows and sum_a D_a v_a in the continuity rows."""
    box = box_of(n, lens)
    X = lattice(box)
    nu, dt = 0.3, 0.7
    x = np.random.default_rng(1).standard_normal((4, box.n_fine))
    lin, _ = odd_even(q2, box, ns_of(nu, dt), X, x)
    M, K, B, D = mats3(box)
    for a in range(3):
        ref = M @ x[a] / dt + 0.5 * nu * (K @ x[a]) - B[a] @ x[3]
        assert rel(lin[a], ref) < 1e-12, a
    ref = sum(D[a] @ x[a] for a in range(3))
    assert rel(lin[3], ref) < 1e-12


def test_q2_convection_by_a_constant_field_is_kronecker(q2):
    """A(c + u) - A(c - u) = 2 Lin(u) + (c.grad u_a, phi) per component:
    sum_d c_d D_d u_a (exact: degree <= 4 per direction)."""
    box = box_of((2, 3, 2), (0.8, 1.1, 0.6))
    X = lattice(box)
    ns = ns_of(0.2, 0.4)
    rng = np.random.default_rng(2)
    u = rng.standard_normal((4, box.n_fine))
    u[3] = 0.0
    c = np.array([0.7, -1.3, 0.4])
    C = np.zeros_like(u)
    C[:3] = c[:, None]
    A1 = q2.apply(box, ns, X, C + u)
    A2 = q2.apply(box, ns, X, C - u)
    lin, _ = odd_even(q2, box, ns, X, u)
    M, K, B, D = mats3(box)
    for a in range(3):
        conv = sum(c[d] * (D[d] @ u[a]) for d in range(3))
        assert rel(0.5 * (A1[a] - A2[a]) - lin[a], 0.5 * conv) < 1e-12


def test_q2_rhs_parts(q2):
    """Rhs(v) = (1/k) M v - 1/2 N(v) - nu/2 K v + M fmid; its odd part is the
    Kronecker form and its even part is minus the even part of A."""
    box = box_of((2, 2, 3), (0.9, 0.8, 1.2))
    X = lattice(box)
    nu, dt = 0.25, 0.6
    ns = ns_of(nu, dt)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((3, box.n_fine))
    f = rng.standard_normal((3, box.n_fine))
    Rp = q2.rhs(box, ns, X, v)
    Rm = q2.rhs(box, ns, X, -v)
    M, K, B, D = mats3(box)
    x = np.concatenate([v, np.zeros((1, box.n_fine))])
    _, even = odd_even(q2, box, ns, X, x)
    for a in range(3):
        assert rel(0.5 * (Rp[a] - Rm[a]), M @ v[a] / dt - 0.5 * nu * (K @ v[a])) < 1e-12
        assert rel(0.5 * (Rp[a] + Rm[a]), -even[a]) < 1e-12
    assert np.all(Rp[3] == 0.0)
    F = q2.rhs(box, ns, X, np.zeros_like(v), fmid=f)
    for a in range(3):
        assert rel(F[a], M @ f[a]) < 1e-12


# ---------------------------------------------------- affine and curved maps --

AFF = np.array([[1.1, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.3]])


def mass_rows(q2, box, X):
    """int phi_i = k (A(e_u))_u with e_u = (1, 0, 0, 0): gradient-free field."""
    x = np.zeros((4, box.n_fine))
    x[0] = 1.0
    return q2.apply(box, ns_of(1.0, 1.0), X, x)[0]


def interior(box):
    idx = syn.lattice_index(box, fine=True)
    m = np.ones(box.n_fine, dtype=bool)
    for a in range(3):
        m &= (idx[a] > 0) & (idx[a] < box.fine_shape[a] - 1)
    return m


def test_q2_affine_mesh_reproduces_polynomials(q2):
    box = box_of((2, 3, 2), (1.0, 0.8, 0.9))
    Y = lattice(box)
    X = AFF @ Y + np.array([0.3, -0.2, 0.5])[:, None]
    inn = interior(box)
    M, _, _, _ = mats3(box)
    m = mass_rows(q2, box, X)
    assert rel(m, np.linalg.det(AFF) * (M @ np.ones(box.n_fine))) < 1e-12

    # stiffness: u quadratic in physical coordinates, -Laplace u constant
    Q = np.array([[0.8, 0.3, -0.1], [0.3, -0.4, 0.2], [-0.1, 0.2, 0.6]])
    u = np.einsum("in,ij,jn->n", X, Q, X) + np.array([0.2, -0.5, 0.1]) @ X
    x = np.zeros((4, box.n_fine))
    x[0] = u
    nu = 2.0
    L1, _ = odd_even(q2, box, ns_of(nu, 0.5), X, x)
    L2, _ = odd_even(q2, box, ns_of(nu, 0.25), X, x)
    Mu = (L1[0] - L2[0]) / (1 / 0.5 - 1 / 0.25)
    Ku = (L1[0] - Mu / 0.5) / (0.5 * nu)
    lap = 2.0 * np.trace(Q)
    assert rel(Ku[inn], -lap * m[inn]) < 1e-11

    # divergence of a linear velocity (every node) and gradient of a linear
    # pressure (interior nodes, after integration by parts)
    W = np.array([[0.4, -0.7, 0.2], [0.5, 0.3, -0.6], [0.1, 0.8, -0.9]])
    g = np.array([0.6, -1.1, 0.35])
    x = np.zeros((4, box.n_fine))
    x[:3] = W @ X
    x[3] = g @ X
    lin, _ = odd_even(q2, box, ns_of(nu, 1e30), X, x)
    assert rel(lin[3], np.trace(W) * m) < 1e-12
    xp = np.zeros_like(x)
    xp[3] = x[3]
    lin, _ = odd_even(q2, box, ns_of(nu, 1e30), X, xp)
    for a in range(3):
        assert rel(lin[a][inn], g[a] * m[inn]) < 1e-11

    # convection: v = c + W x with W^2 = 0, so v.grad v = W c everywhere
    Wn = np.zeros((3, 3))
    Wn[0, 1] = 0.9
    Wn[0, 2] = -0.4
    c = np.array([0.3, 1.2, -0.7])
    x = np.zeros((4, box.n_fine))
    x[:3] = c[:, None] + Wn @ X
    _, even = odd_even(q2, box, ns_of(nu, 1.0), X, x)
    wc = Wn @ c
    for a in range(3):
        assert np.allclose(even[a], 0.5 * wc[a] * m, rtol=0, atol=1e-13 * np.abs(m).max() + 1e-15)


def quad_map(Y, eps):
    """A global quadratic map X = Y + eps g(Y) (exactly Q2 on every element)."""
    y0, y1, y2 = Y
    g = np.stack([y1 * y2 - 0.5 * y0 * y1, y0 * y0 - 0.3 * y2 * y2 + y0 * y2, 0.4 * y0 * y1 - y1 * y1])
    return Y + eps * g


def quad_map_jac_det(y, eps):
    y0, y1, y2 = y
    J = np.zeros((3, 3) + y0.shape)
    J[0, 0] = 1 - 0.5 * eps * y1
    J[0, 1] = eps * (y2 - 0.5 * y0)
    J[0, 2] = eps * y1
    J[1, 0] = eps * (2 * y0 + y2)
    J[1, 1] = 1.0
    J[1, 2] = eps * (-0.6 * y2 + y0)
    J[2, 0] = 0.4 * eps * y1
    J[2, 1] = eps * (0.4 * y0 - 2 * y1)
    J[2, 2] = 1.0
    return np.linalg.det(np.moveaxis(J, (0, 1), (-2, -1)))


def test_q2_isoparametric_volume_and_linear_fields(q2):
    """Curved elements: det J of a global quadratic map has total degree 3,
    so the 3-point rule integrates it exactly; linear physical fields lie in
    the isoparametric space, so their gradients are exact."""
    box = box_of((2, 2, 3), (1.0, 0.9, 1.2))
    Y = lattice(box)
    eps = 0.25
    X = quad_map(Y, eps)
    assert q2.min_det(box, X) > 0
    m = mass_rows(q2, box, X)
    # independent volume: 4-point Gauss-Legendre over the reference box
    t, w = np.polynomial.legendre.leggauss(4)
    pts = [0.5 * L * (t + 1) for L in box.len]
    wts = [0.5 * L * w for L in box.len]
    G = np.meshgrid(*pts, indexing="ij")
    Wt = np.einsum("i,j,k->ijk", *wts)
    vol = float(np.sum(Wt * quad_map_jac_det(np.stack(G), eps)))
    assert abs(m.sum() - vol) < 1e-12 * vol
    W = np.array([[0.4, -0.7, 0.2], [0.5, 0.3, -0.6], [0.1, 0.8, -0.9]])
    x = np.zeros((4, box.n_fine))
    x[:3] = W @ X
    lin, _ = odd_even(q2, box, ns_of(1.0, 1e30), X, x)
    assert rel(lin[3], np.trace(W) * m) < 1e-12


def rot(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def test_q2_rigid_motion_equivariance(q2):
    """All terms, LPS included, on a distorted mesh: A(R X + t; R v, p) =
    (R A_v, A_p)."""
    box = syn.channel_box((4, 2, 2))
    X = syn.distorted_coords(box, amp=0.2, seed=3)
    ns = syn.NSParams(2e-3, 0.01, 0.02, 0.1)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((4, box.n_fine))
    A = q2.apply(box, ns, X, x)
    R = rot(5)
    xr = x.copy()
    xr[:3] = R @ x[:3]
    Ar = q2.apply(box, ns, R @ X + np.array([1.0, -2.0, 0.5])[:, None], xr)
    assert rel(Ar[:3], R @ A[:3]) < 1e-12
    assert rel(Ar[3], A[3]) < 1e-12


# ------------------------------------------------------------- LPS terms ----

def elementwise_q1(box, vals):
    """Fields [c][N] that are Q1 on every element: vertex values (all lattice
    indices even) as given, every other node the mean of the element's
    vertices around it (the trilinear interpolant at reference midpoints)."""
    idx = syn.lattice_index(box, fine=True)
    Nf = box.fine_shape
    out = vals.copy()
    for n in range(box.n_fine):
        i = idx[:, n]
        odd = [a for a in range(3) if i[a] % 2]
        if not odd:
            continue
        acc = 0.0
        cnt = 0
        for s in range(1 << len(odd)):
            j = i.copy()
            for t, a in enumerate(odd):
                j[a] += 1 if (s >> t) & 1 else -1
            acc = acc + vals[:, j[0] + Nf[0] * (j[1] + Nf[1] * j[2])]
            cnt += 1
        out[:, n] = acc / cnt
    return out


def test_q2_lps_vanishes_on_elementwise_q1_fields(q2):
    box = syn.channel_box((4, 2, 2))
    box.dirichlet_mask = 0
    X = syn.distorted_coords(box, amp=0.2, seed=6)
    x = elementwise_q1(box, np.random.default_rng(7).standard_normal((4, box.n_fine)))
    on = q2.apply(box, syn.NSParams(2e-3, 0.01, 0.5, 0.7), X, x)
    off = q2.apply(box, syn.NSParams(2e-3, 0.01, 0.0, 0.0), X, x)
    assert rel(on, off) < 1e-13
    # and they do not vanish on a general field
    y = np.random.default_rng(8).standard_normal((4, box.n_fine))
    on = q2.apply(box, syn.NSParams(2e-3, 0.01, 0.5, 0.7), X, y)
    off = q2.apply(box, syn.NSParams(2e-3, 0.01, 0.0, 0.0), X, y)
    assert rel(on, off) > 1e-3


NU, DT = 0.6, 0.8
LPS_BOX = ((2, 2, 2), (0.9, 0.7, 1.3))


def elem_ops(box):
    """Per-element 27 x 27 stiffness, streamline matrices and I - Pi_T."""
    H = [box.len[a] / box.n[a] for a in range(3)]
    e = [elem1d(H[a]) for a in range(3)]

    def k3(a, b, c):  # local node a + 3b + 9c: x fastest
        return np.kron(c, np.kron(b, a))

    K = (k3(e[0]["K"], e[1]["M"], e[2]["M"]) + k3(e[0]["M"], e[1]["K"], e[2]["M"])
         + k3(e[0]["M"], e[1]["M"], e[2]["K"]))
    P1 = np.array([[1.0, 0.0, 0.0], [0.5, 0.0, 0.5], [0.0, 0.0, 1.0]])
    IP = np.eye(27) - k3(P1, P1, P1)

    def S(c):
        # S[i, j] = sum_de c_d c_e int d_d phi_j d_e phi_i (row = test function)
        out = np.zeros((27, 27))
        for d in range(3):
            for f in range(3):
                F = []
                for a in range(3):
                    if a == d and a == f:
                        F.append(e[a]["K"])
                    elif a == d:
                        F.append(e[a]["C"].T)    # int phi_j' phi_i
                    elif a == f:
                        F.append(e[a]["C"])      # int phi_i' phi_j
                    else:
                        F.append(e[a]["M"])
                out += c[d] * c[f] * k3(*F)
        return out

    hT = float(np.sqrt(sum(h * h for h in H)))
    return K, IP, S, hT


def elem_nodes(box, I, J, K):
    Nf = box.fine_shape
    return np.array([(2 * I + a) + Nf[0] * ((2 * J + b) + Nf[1] * (2 * K + c))
                     for c in range(3) for b in range(3) for a in range(3)])


def lps_assemble(box, Mloc):
    out = sp.lil_matrix((box.n_fine, box.n_fine))
    for K in range(box.n[2]):
        for J in range(box.n[1]):
            for I in range(box.n[0]):
                g = elem_nodes(box, I, J, K)
                for i in range(27):
                    for j in range(27):
                        out[g[i], g[j]] += Mloc[i, j]
    return out.tocsr()


def alpha_pin(q2, L=None):
    box = box_of(*LPS_BOX)
    X = lattice(box)
    Kl, IP, S, hT = elem_ops(box)
    c = np.array([0.6, -0.8, 0.5])
    a0 = 0.7
    rng = np.random.default_rng(11)
    x = np.zeros((4, box.n_fine))
    x[:3] = c[:, None]
    x[3] = rng.standard_normal(box.n_fine)
    on = q2.apply(box, syn.NSParams(NU, DT, a0, 0.0), X, x, L=L)
    off = q2.apply(box, syn.NSParams(NU, DT, 0.0, 0.0), X, x, L=L)
    den = NU / hT ** 2 + np.linalg.norm(c) / hT + 1 / DT
    ref = (a0 / den) * (lps_assemble(box, IP.T @ Kl @ IP) @ x[3])
    return rel(on[3] - off[3], ref)


def delta_pin(q2, L=None):
    box = box_of(*LPS_BOX)
    X = lattice(box)
    Kl, IP, S, hT = elem_ops(box)
    c = np.array([0.9, 0.4, -0.3])
    d0 = 0.6
    rng = np.random.default_rng(12)
    # u perpendicular to c with |u| = 1 at every node
    u = rng.standard_normal((3, box.n_fine))
    ch = c / np.linalg.norm(c)
    u -= ch[:, None] * (ch @ u)
    u /= np.linalg.norm(u, axis=0)

    def odd(eps):
        def A(s, dd):
            x = np.zeros((4, box.n_fine))
            x[:3] = c[:, None] + s * eps * u
            return q2.apply(box, syn.NSParams(NU, DT, 0.0, dd), X, x, L=L)
        return ((A(1, d0) - A(1, 0.0)) - (A(-1, d0) - A(-1, 0.0))) / (2 * eps)

    e = 1e-3
    lin = (4 * odd(e) - odd(2 * e)) / 3
    den = NU / hT ** 2 + np.linalg.norm(c) / hT + 1 / DT
    Sg = lps_assemble(box, IP.T @ S(c) @ IP)
    ref = np.stack([(d0 / den) * (Sg @ u[a]) for a in range(3)])
    return rel(lin[:3], ref)


def test_q2_alpha_term_magnitude(q2):
    assert alpha_pin(q2) < 1e-12


def test_q2_delta_term_magnitude(q2):
    assert delta_pin(q2) < 1e-9


def test_q2_stabilisation_terms_all_weigh():
    box = box_of(*LPS_BOX)
    _, _, _, hT = elem_ops(box)
    terms = [NU / hT ** 2, 1.0 / hT, 1 / DT]
    assert min(terms) / sum(terms) > 0.1


SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "q2_oracle.c")
MUTATIONS = {
    "h_T shortest edge": ("if (sqrt(d2) > hT) hT = sqrt(d2);",
                          "if ((v ^ w) == 1 || (v ^ w) == 2 || (v ^ w) == 4) { if (hT == 0.0 || sqrt(d2) < hT) hT = sqrt(d2); }"),
    "nu term dropped": ("double den = ns->nu / (hT * hT) + vmax / hT + 1.0 / ns->dt;",
                        "double den = vmax / hT + 1.0 / ns->dt;"),
    "nu / h_T": ("double den = ns->nu / (hT * hT) + vmax / hT + 1.0 / ns->dt;",
                 "double den = ns->nu / hT + vmax / hT + 1.0 / ns->dt;"),
    "|v| / h_T^2": ("double den = ns->nu / (hT * hT) + vmax / hT + 1.0 / ns->dt;",
                    "double den = ns->nu / (hT * hT) + vmax / (hT * hT) + 1.0 / ns->dt;"),
    "1/k dropped": ("double den = ns->nu / (hT * hT) + vmax / hT + 1.0 / ns->dt;",
                    "double den = ns->nu / (hT * hT) + vmax / hT;"),
    "alpha term halved": ("alphaT = ns->alpha0 / den;", "alphaT = 0.5 * ns->alpha0 / den;"),
    "delta term doubled": ("deltaT = ns->delta0 / den;", "deltaT = 2.0 * ns->delta0 / den;"),
    "pi phi of vertices dropped": ("if (vof[i] >= 0)", "if (0)"),
}


@contextlib.contextmanager
def altered(q2, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "m.c")
        so = os.path.join(tmp, "m.so")
        open(c, "w").write(src.replace(old, new))
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", c, "-o", so, "-lm"])
        yield q2.load(so)


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_q2_altered_stabilisation_fails_a_pin(q2, name):
    old, new = MUTATIONS[name]
    with altered(q2, old, new) as L:
        worst = max(alpha_pin(q2, L), delta_pin(q2, L))
    assert worst > 1e-6, name


# -------------------------------------------------------------- transfer ----

def test_q2_prolongation_reproduces_quadratics(q2):
    box = box_of((4, 2, 6), (1.0, 0.5, 1.5))
    Yf = syn.node_coords(box, fine=True)
    Yc = syn.node_coords(box, fine=False)

    def f(P):
        y0, y1, y2 = P
        return np.stack([1 + y0 - 2 * y1 * y2 + 3 * y0 * y0, y1 * y1 - y0 * y2 + 0.5, y2 - y0 * y1])

    xf = q2.prolong(box, f(Yc))
    assert np.abs(xf - f(Yf)).max() < 1e-13
    # a cubic is not reproduced (the interpolation is of degree 2)
    assert np.abs(q2.prolong(box, Yc[0:1] ** 3) - Yf[0:1] ** 3).max() > 1e-4


def test_q2_restriction_is_the_transpose(q2):
    box = box_of((2, 4, 2))
    rng = np.random.default_rng(13)
    xc = rng.standard_normal((2, box.n_coarse))
    yf = rng.standard_normal((2, box.n_fine))
    assert abs(np.sum(q2.prolong(box, xc) * yf) - np.sum(xc * q2.restrict(box, yf))) < 1e-12 * np.abs(yf).sum()


def test_q2_galerkin_identity_of_the_linear_terms(q2):
    """R Lin_fine(P x) = Lin_coarse(x) on an affine mesh (both quadratures
    exact for the linear terms), coarse nodes = the fine nodes with even
    indices."""
    fine = box_of((4, 2, 2), (1.0, 0.6, 0.8))
    coarse = box_of((2, 1, 1), (1.0, 0.6, 0.8))
    Xf = AFF @ lattice(fine)
    Xc = AFF @ lattice(coarse)
    idx = syn.lattice_index(fine, fine=True)
    even = np.all(idx % 2 == 0, axis=0)
    assert np.allclose(Xf[:, even], Xc)
    ns = ns_of(0.3, 0.45)
    x = np.random.default_rng(14).standard_normal((4, coarse.n_fine))
    lf, _ = odd_even(q2, fine, ns, Xf, q2.prolong(fine, x))
    lc, _ = odd_even(q2, coarse, ns, Xc, x)
    assert rel(q2.restrict(fine, lf), lc) < 1e-12


# ----------------------------------------------------------------- gather --

def test_q2_gather_brute_force(q2):
    box = syn.channel_box((2, 2, 2))
    X = syn.distorted_coords(box, amp=0.2, seed=15)
    rng = np.random.default_rng(16)
    x = rng.standard_normal((4, box.n_fine))
    r = rng.standard_normal((4, box.n_fine))
    shift = rng.standard_normal(165)
    inv = rng.uniform(0.5, 2.0, 165)
    G = q2.gather(box, X, x, r, shift, inv)
    Nf = box.fine_shape
    for K in range(2):
        for J in range(2):
            for I in range(2):
                M = I + 2 * (J + 2 * K)
                nodes = [(2 * I + a) + Nf[0] * ((2 * J + b) + Nf[1] * (2 * K + c))
                         for c in range(3) for b in range(3) for a in range(3)]
                verts = [(2 * I + 2 * a) + Nf[0] * ((2 * J + 2 * b) + Nf[1] * (2 * K + 2 * c))
                         for c in range(2) for b in range(2) for a in range(2)]
                feat = []
                for ax in range(3):
                    ls = []
                    for v in range(8):
                        if (v >> ax) & 1 == 0:
                            w = v | (1 << ax)
                            ls.append(np.linalg.norm(X[:, verts[w]] - X[:, verts[v]]))
                    feat.append(np.mean(ls))
                row = np.concatenate([x[0, nodes], x[1, nodes], x[2, nodes], r[0, nodes], r[1, nodes],
                                      r[2, nodes], feat])
                assert np.allclose(G[M], (row - shift) * inv, rtol=1e-14, atol=1e-14)
    # on the lattice the geometry inputs are the element sizes
    Xl = lattice(box)
    F = q2.features(box, Xl)
    assert np.allclose(F, np.array([box.len[a] / box.n[a] for a in range(3)])[None, :])


def test_q2_dirichlet_rows_and_residual_form(q2):
    box = syn.channel_box((2, 2, 2))
    X = syn.distorted_coords(box, amp=0.2, seed=17)
    ns = syn.NSParams(1e-3, 0.005)
    rng = np.random.default_rng(18)
    x = rng.standard_normal((4, box.n_fine))
    vp = rng.standard_normal((3, box.n_fine))
    r = q2.residual(box, ns, X, x, vp)
    dm = syn.boundary_mask(box, fine=True)
    assert np.all(r[:3, dm] == 0.0)
    full = q2.rhs(box, ns, X, vp) - q2.apply(box, ns, X, x)
    assert np.allclose(r[:, ~dm], full[:, ~dm], rtol=0, atol=1e-12 * np.abs(full).max())
    assert np.abs(r[3, dm]).max() > 0
