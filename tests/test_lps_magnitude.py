"""Magnitude pins of the two local projection terms of eq. (disc:ns) and of the
stabilisation parameters of eq. (stabparams).

The projection pi of the two-level stabilisation is interpolation onto the Q1
space of each patch (coarse cell), so on every fine field f the fluctuation
f - pi f is (I - P Inj) f, with Inj the injection at the coarse vertices and
P the Q1 prolongation.  Both LPS terms are then bilinear forms of textbook
Kronecker stencils applied to the fluctuations:

  alpha term (continuity rows, any constant velocity c):
      r_p(alpha0) - r_p(0) = -alpha_T (I - P Inj)^T K (I - P Inj) p
  delta term (momentum rows, v = c + eps u with u perpendicular to c and
  |u| = 1 at every node, so |v| = sqrt(|c|^2 + eps^2) on every cell): the
  part of r_a(delta0) - r_a(0) that is linear in eps is
      -delta_T (I - P Inj)^T S_c (I - P Inj) u_a,
      S_c[i, j] = int (c . grad phi_j)(c . grad phi_i),
with alpha_T = alpha0 / den, delta_T = delta0 / den, den = nu / h_T^2 +
|v|_inf,T / h_T + 1 / k and h_T the cell diameter.  K and the entries of S_c are
Kronecker products of the 1-D Q1 mass, stiffness and first-derivative
matrices (exact under the 2-point Gauss rule on rectangles).  Parameters are
chosen so that each of the three terms of den carries weight.

The second half compiles altered copies of the oracle (h_T as the shortest
edge, each term of den changed, either LPS term scaled) and checks that every
alteration fails at least one of the two pins.
"""
import contextlib
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.sparse as sp

import dnnmg_synth as syn
from test_oracle_pins import fine_mats, kron3, prolong1d

NU, DT = 0.15, 0.5


def boxes():
    return [syn.BoxSpec((2, 2, 2), (1.0, 0.6, 1.4), 7, 0),   # periodic, anisotropic cells
            syn.BoxSpec((2, 2, 2), (0.9, 0.7, 1.3), 0, 0)]   # open axes, no Dirichlet rows


def interp_fluctuation(box):
    """I - P Inj on the fine nodes (Kronecker products of 1-D operators)."""
    per = [(box.periodic_mask >> a) & 1 for a in range(3)]
    Ps, Is = [], []
    for a in range(3):
        P1 = prolong1d(box.n[a], per[a])
        nf1, nc1 = P1.shape
        I1 = sp.lil_matrix((nc1, nf1))
        for I in range(nc1):
            I1[I, 2 * I] = 1.0
        Ps.append(P1)
        Is.append(I1.tocsr())
    Pi = kron3(*Ps) @ kron3(*Is)
    return (sp.identity(box.n_fine, format="csr") - Pi).tocsr()


def stiffness(box):
    m = fine_mats(box)
    Mx, My, Mz = m["M"]; Kx, Ky, Kz = m["K"]
    return kron3(Kx, My, Mz) + kron3(Mx, Ky, Mz) + kron3(Mx, My, Kz)


def streamline(box, c):
    """S_c[i, j] = sum_de c_d c_e int d_d phi_j d_e phi_i (row = test function)."""
    m = fine_mats(box)
    S = None
    for d in range(3):
        for e in range(3):
            F = []
            for a in range(3):
                if a == d and a == e:
                    F.append(m["K"][a])
                elif a == d:
                    F.append(m["C"][a])          # int phi_j' phi_i
                elif a == e:
                    F.append(m["C"][a].T)        # int phi_j phi_i'
                else:
                    F.append(m["M"][a])
            t = c[d] * c[e] * kron3(*F)
            S = t if S is None else S + t
    return S.tocsr()


def cell_params(box, vnorm, a0, d0):
    h = np.array([box.len[a] / (2 * box.n[a]) for a in range(3)])
    hT = float(np.sqrt(np.sum(h * h)))           # cell diameter
    den = NU / hT ** 2 + vnorm / hT + 1.0 / DT
    return a0 / den, d0 / den


def alpha_pin(orc, box):
    """Largest relative deviation of the alpha term from its Kronecker form,
    over v = 0 and a constant v."""
    nf = box.n_fine
    Q = interp_fluctuation(box)
    K = stiffness(box)
    rng = np.random.default_rng(21)
    worst = 0.0
    for c in (np.zeros(3), np.array([0.7, -0.4, 0.5])):
        x = np.zeros((4, nf))
        x[:3] = c[:, None]
        x[3] = rng.standard_normal(nf)
        on = orc.residual(box, syn.NSParams(NU, DT, 0.3, 0.0), x, x[:3].copy())
        off = orc.residual(box, syn.NSParams(NU, DT, 0.0, 0.0), x, x[:3].copy())
        alphaT, _ = cell_params(box, float(np.linalg.norm(c)), 0.3, 0.0)
        want = -alphaT * (Q.T @ (K @ (Q @ x[3])))
        got = on[3] - off[3]
        worst = max(worst, float(np.abs(got - want).max() / np.abs(want).max()))
    return worst


def delta_pin(orc, box):
    """Largest relative deviation of the eps-linear part of the delta term
    from its Kronecker form, per momentum component."""
    nf = box.n_fine
    Q = interp_fluctuation(box)
    c = np.array([0.8, 0.35, -0.6])
    S = streamline(box, c)
    rng = np.random.default_rng(22)
    u = rng.standard_normal((3, nf))
    chat = c / np.linalg.norm(c)
    u -= chat[:, None] * (chat @ u)[None, :]
    u /= np.linalg.norm(u, axis=0)[None, :]
    vp = rng.standard_normal((3, nf))

    def odd(eps):
        # (L(eps) - L(-eps)) / (-2 delta_T) = eps A + eps^3 C exactly
        parts = []
        for s in (eps, -eps):
            x = np.zeros((4, nf))
            x[:3] = c[:, None] + s * u
            on = orc.residual(box, syn.NSParams(NU, DT, 0.0, 0.2), x, vp)
            off = orc.residual(box, syn.NSParams(NU, DT, 0.0, 0.0), x, vp)
            parts.append(on[:3] - off[:3])
        _, dT = cell_params(box, float(np.sqrt(c @ c + eps * eps)), 0.0, 0.2)
        return (parts[0] - parts[1]) / (-2.0 * dT)

    e1, e2 = 0.25, 0.5
    A = (e2 ** 3 * odd(e1) - e1 ** 3 * odd(e2)) / (e1 * e2 ** 3 - e2 * e1 ** 3)
    worst = 0.0
    for a in range(3):
        want = Q.T @ (S @ (Q @ u[a]))
        worst = max(worst, float(np.abs(A[a] - want).max() / np.abs(want).max()))
    return worst


@pytest.mark.parametrize("box", boxes(), ids=["periodic", "open"])
def test_lps_alpha_term_magnitude(orc, box):
    assert alpha_pin(orc, box) <= 1e-12


@pytest.mark.parametrize("box", boxes(), ids=["periodic", "open"])
def test_lps_delta_term_magnitude(orc, box):
    assert delta_pin(orc, box) <= 1e-12


def test_stabilisation_terms_all_weigh():
    """The pins only see what carries weight: every term of den is at least
    10 % of den for these parameters, and the cell diameter differs from the
    shortest edge."""
    for box in boxes():
        h = np.array([box.len[a] / (2 * box.n[a]) for a in range(3)])
        hT = np.sqrt(np.sum(h * h))
        for vnorm in (np.linalg.norm([0.7, -0.4, 0.5]), np.linalg.norm([0.8, 0.35, -0.6])):
            terms = np.array([NU / hT ** 2, vnorm / hT, 1.0 / DT])
            assert terms.min() >= 0.1 * terms.sum()
        assert hT > 1.5 * h.min()


# ----------------------------------------------------- altered oracles -------

HT_LINE = "double hT = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);"
DEN_LINE = "double den = ns->nu / (hT * hT) + vmax / hT + 1.0 / ns->dt;"
ALPHA_LINE = "alphaT = ns->alpha0 / den;"
DELTA_LINE = "deltaT = ns->delta0 / den;"

MUTATIONS = {
    "h_T shortest edge": (HT_LINE, "double hT = fmin(h[0], fmin(h[1], h[2]));"),
    "h_T longest edge": (HT_LINE, "double hT = fmax(h[0], fmax(h[1], h[2]));"),
    "nu/h_T^2 dropped": (DEN_LINE, "double den = vmax / hT + 1.0 / ns->dt;"),
    "nu/h_T instead of nu/h_T^2": (DEN_LINE, "double den = ns->nu / hT + vmax / hT + 1.0 / ns->dt;"),
    "|v|/h_T dropped": (DEN_LINE, "double den = ns->nu / (hT * hT) + 1.0 / ns->dt;"),
    "|v|/h_T^2": (DEN_LINE, "double den = ns->nu / (hT * hT) + vmax / (hT * hT) + 1.0 / ns->dt;"),
    "1/k dropped": (DEN_LINE, "double den = ns->nu / (hT * hT) + vmax / hT;"),
    "alpha term doubled": (ALPHA_LINE, "alphaT = 2.0 * ns->alpha0 / den;"),
    "delta term halved": (DELTA_LINE, "deltaT = 0.5 * ns->delta0 / den;"),
}


@contextlib.contextmanager
def altered_oracle(orc, old, new, tmp):
    src = open(os.path.join(os.path.dirname(orc.__file__), "dnnmg_oracle.c")).read()
    # the stabilisation parameters of the residual come first in the file
    assert old in src
    src = src.replace(old, new, 1)
    path_c = os.path.join(tmp, "oracle_altered.c")
    path_so = os.path.join(tmp, f"liboracle_altered_{abs(hash(new))}.so")
    open(path_c, "w").write(src)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", path_c, "-o",
                           path_so, "-lm"])
    saved = orc.lib()
    orc._lib = orc.load(path_so)
    try:
        yield
    finally:
        orc._lib = saved


def test_pinned_lines_are_in_the_oracle(orc):
    src = open(os.path.join(os.path.dirname(orc.__file__), "dnnmg_oracle.c")).read()
    for line in (HT_LINE, DEN_LINE, ALPHA_LINE, DELTA_LINE):
        assert line in src


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_altered_stabilisation_fails_a_pin(orc, name):
    old, new = MUTATIONS[name]
    with tempfile.TemporaryDirectory() as tmp, altered_oracle(orc, old, new, tmp):
        errs = [f(orc, box) for box in boxes() for f in (alpha_pin, delta_pin)]
    assert max(errs) > 1e-6, (name, errs)
