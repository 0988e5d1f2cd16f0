"""Plain FP64 Crank-Nicolson solves on one mesh level (test infrastructure).

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): the judge of the
correction and the source of the teacher-forced training pairs used by the
tests.  Newton's method on the discrete system (Sec. 2.4: the Jacobian is
kept across iterations and time steps and re-assembled only when the
contraction rate of the residual exceeds rho_max), with the Jacobian
assembled column-wise by central finite differences of the oracle residual
(nodes coloured with period 5 per axis: the residual of a node depends on
nodes at most 2 lattice steps away) and solved by sparse LU (scipy).
Non-periodic boxes only (the pressure is then determined).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dirichlet_flags, fine_nodes, prolong, residual, restrict, rhs


def _lattice(box):
    nx, ny, nz = [2 * box.n[a] + 1 for a in range(3)]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel(), (nx, ny, nz)


def fd_jacobian(box, ns, x, h=1e-6):
    """J = -d r / d x of the fine residual of `box` (a sparse 4 N x 4 N
    matrix), Dirichlet velocity rows replaced by identity rows."""
    assert box.periodic_mask == 0, "non-periodic boxes only"
    nf = fine_nodes(box)
    i, j, k, (nx, ny, nz) = _lattice(box)
    colour = (i % 5) + 5 * (j % 5) + 25 * (k % 5)
    zero_vp = np.zeros((3, nf))
    rows, cols, vals = [], [], []
    x = np.asarray(x, dtype=np.float64).reshape(4, nf)
    for f in range(4):
        for c in range(125):
            sel = np.where(colour == c)[0]
            if sel.size == 0:
                continue
            e = np.zeros((4, nf))
            e[f, sel] = h
            dr = -(residual(box, ns, x + e, zero_vp) - residual(box, ns, x - e, zero_vp)) / (2 * h)
            # each coloured node owns the rows within 2 lattice steps
            for n in sel:
                di = np.abs(i - i[n]) <= 2
                dj = np.abs(j - j[n]) <= 2
                dk = np.abs(k - k[n]) <= 2
                near = np.where(di & dj & dk)[0]
                for g in range(4):
                    v = dr[g, near]
                    nz_ = v != 0.0
                    rows.append(g * nf + near[nz_])
                    cols.append(np.full(int(nz_.sum()), f * nf + n))
                    vals.append(v[nz_])
    J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(4 * nf, 4 * nf))
    dmask = dirichlet_flags(box).astype(bool)
    keep = np.ones(4 * nf)
    for f in range(3):
        keep[f * nf + np.where(dmask)[0]] = 0.0
    D = sp.diags(keep)
    J = (D @ J + sp.diags(1.0 - keep)).tocsc()
    return J


class NewtonSolver:
    """Newton iterations on R(x) = 0 with a lazily re-assembled Jacobian."""

    def __init__(self, box, ns, rho_max=0.1):
        self.box, self.ns, self.rho_max = box, ns, rho_max
        self.lu = None
        self.assemblies = 0

    def _factor(self, x):
        self.lu = spla.splu(fd_jacobian(self.box, self.ns, x))
        self.assemblies += 1

    def solve(self, R, x0, rtol=1e-10, atol=1e-13, maxit=30):
        """R(x) returns the residual [4][N] (b - A(x)); Dirichlet rows zero."""
        x = np.array(x0, dtype=np.float64)
        r = R(x)
        r0 = np.linalg.norm(r)
        if self.lu is None:
            self._factor(x)
        for it in range(maxit):
            nr = np.linalg.norm(r)
            if nr <= max(rtol * r0, atol):
                return x, it
            dx = self.lu.solve(r.ravel()).reshape(x.shape)
            x = x + dx
            r_new = R(x)
            if np.linalg.norm(r_new) > self.rho_max * nr:
                self._factor(x)  # slow contraction: new Jacobian at the current iterate
            r = r_new
        raise RuntimeError(f"Newton did not converge: |r| = {np.linalg.norm(r):.3e} (r0 = {r0:.3e})")


def coarse_box_of(box):
    """The coarse level of `box` as a box whose fine mesh is that level."""
    assert all(n % 2 == 0 for n in box.n), "coarse level needs even cell counts"
    return type(box)(tuple(n // 2 for n in box.n), box.len, box.periodic_mask, box.dirichlet_mask)


def teacher_forced(box, ns, vbar0, xc0, steps, fine_bc, coarse_bc, log=None):
    """Teacher-forced pairs of the plain method (a reading of Sec. 4.2):
      F_n   = Rhs_fine(vbar_{n-1})                     (Algorithm 1, Rhs)
      x^L_n : A_coarse(x^L_n) = R F_n                   (coarse solve)
      xbar_n: A_fine(xbar_n) = F_n                      (fine solve, ground truth)
    fine_bc / coarse_bc: (mask over [4][N], values) of the Dirichlet data.
    Returns lists xc[n] (coarse solutions), vbar[n] (fine velocities,
    vbar[0] = initial) and the fine pressures."""
    cbox = coarse_box_of(box)
    nf = fine_nodes(box)
    fine = NewtonSolver(box, ns)
    coarse = NewtonSolver(cbox, ns)
    vbar = [np.asarray(vbar0, dtype=np.float64).reshape(3, nf)]
    pbar = [np.zeros(nf)]
    xcs = []
    xc = np.asarray(xc0, dtype=np.float64)
    cmask = dirichlet_flags(cbox).astype(bool)
    for n in range(1, steps + 1):
        vp = vbar[-1]
        F = rhs(box, ns, vp)
        bL = restrict(box, F)
        bL[:3, cmask] = 0.0
        zero_c = np.zeros((3, bL.shape[1]))
        xc = np.where(coarse_bc[0], coarse_bc[1], xc)
        xc, _ = coarse.solve(lambda z: bL + residual(cbox, ns, z, zero_c), xc)
        x0 = np.concatenate([vp, pbar[-1][None]])
        x0 = np.where(fine_bc[0], fine_bc[1], x0)
        xb, _ = fine.solve(lambda z: residual(box, ns, z, vp), x0)
        xcs.append(xc)
        vbar.append(xb[:3])
        pbar.append(xb[3])
        if log:
            log(f"step {n}: fine Jacobians {fine.assemblies}, coarse {coarse.assemblies}")
    return xcs, vbar, pbar
