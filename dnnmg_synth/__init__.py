"""Seeded synthetic inputs shared by the oracle-side and GPU-side tests.

This module holds workload descriptions and random-number draws only; none of
the method's arithmetic (no prolongation, residual, network or averaging).
Both sides receive the same arrays and apply their own operators to them.

Workloads (sizes follow the project's five configurations):
  * ``cfg1``  unit periodic cube, 4^3 coarse cells, Fourier velocity, MLP width 128
  * ``cfg2``  channel 2.5 x 0.41 x 0.41, 64x16x16 coarse cells, width 256, BF16
  * ``cfg3``  32 periodic unit boxes with uneven even-sized coarse meshes, width 256
  * ``cfg4``  channel 48x12x12 coarse cells, training workload, width 256
  * ``cfg5``  channel 128x32x32 coarse cells, width 512, FP8

The channel stands in for the paper's 3D flow around a cylinder (Sec. 5.2):
same cross-section H = 0.41, a parabolic inflow of peak 1.5 and O(1)
velocities; the obstacle meshes and flow data are not available.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np

# face bits: 2a = low face of axis a, 2a+1 = high face
X_LO, X_HI, Y_LO, Y_HI, Z_LO, Z_HI = 1, 2, 4, 8, 16, 32
CHANNEL_DIRICHLET = X_LO | Y_LO | Y_HI | Z_LO | Z_HI  # inflow + walls, do-nothing outflow
CHANNEL_LEN = (2.5, 0.41, 0.41)
U_MAX = 1.5


@dataclasses.dataclass
class BoxSpec:
    n: Tuple[int, int, int]
    len: Tuple[float, float, float]
    periodic_mask: int
    dirichlet_mask: int

    def fine_axis_nodes(self, a: int) -> int:
        return 2 * self.n[a] if (self.periodic_mask >> a) & 1 else 2 * self.n[a] + 1

    def coarse_axis_nodes(self, a: int) -> int:
        return self.n[a] if (self.periodic_mask >> a) & 1 else self.n[a] + 1

    @property
    def fine_shape(self):
        return tuple(self.fine_axis_nodes(a) for a in range(3))

    @property
    def coarse_shape(self):
        return tuple(self.coarse_axis_nodes(a) for a in range(3))

    @property
    def n_fine(self) -> int:
        s = self.fine_shape
        return s[0] * s[1] * s[2]

    @property
    def n_coarse(self) -> int:
        s = self.coarse_shape
        return s[0] * s[1] * s[2]

    @property
    def n_patches(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


@dataclasses.dataclass
class NSParams:
    nu: float
    dt: float
    alpha0: float = 0.02  # eq. (stabparams)
    delta0: float = 0.1


@dataclasses.dataclass
class Workload:
    name: str
    box: BoxSpec
    ns: NSParams
    hidden: int
    precision: str  # "fp32" | "bf16" | "fp8"
    kind: str       # "fourier" | "channel"


def cfg1() -> Workload:
    return Workload("cfg1_periodic_4x4x4", BoxSpec((4, 4, 4), (1.0, 1.0, 1.0), 7, 0),
                    NSParams(1e-3, 0.01), 128, "fp32", "fourier")


def channel_box(n) -> BoxSpec:
    return BoxSpec(tuple(int(v) for v in n), CHANNEL_LEN, 0, CHANNEL_DIRICHLET)


def cfg2() -> Workload:
    return Workload("cfg2_channel_64x16x16", channel_box((64, 16, 16)), NSParams(1e-3, 0.005),
                    256, "bf16", "channel")


def cfg4() -> Workload:
    return Workload("cfg4_channel_48x12x12", channel_box((48, 12, 12)), NSParams(1e-3, 0.005),
                    256, "bf16", "channel")


def cfg5() -> Workload:
    return Workload("cfg5_channel_128x32x32", channel_box((128, 32, 32)), NSParams(1e-3, 0.005),
                    512, "fp8", "channel")


def cfg3_boxes(seed: int = 0, count: int = 32) -> List[BoxSpec]:
    """Uneven periodic unit boxes: nx even in 8..48, ny, nz in {8, 10, 12}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nx = int(rng.integers(4, 25)) * 2
        ny = int(rng.choice([8, 10, 12]))
        nz = int(rng.choice([8, 10, 12]))
        out.append(BoxSpec((nx, ny, nz), (1.0, 1.0, 1.0), 7, 0))
    return out


def small_channel(n=(4, 2, 2)) -> Workload:
    return Workload("channel_small", channel_box(n), NSParams(1e-3, 0.005), 32, "fp32", "channel")


# ------------------------------------------------------------------ lattices --

def node_coords(box: BoxSpec, fine: bool) -> np.ndarray:
    """Physical coordinates [3][N] of the fine or coarse lattice (x fastest)."""
    shape = box.fine_shape if fine else box.coarse_shape
    h = [box.len[a] / ((2 if fine else 1) * box.n[a]) for a in range(3)]
    k, j, i = np.meshgrid(np.arange(shape[2]), np.arange(shape[1]), np.arange(shape[0]),
                          indexing="ij")
    return np.stack([i.ravel() * h[0], j.ravel() * h[1], k.ravel() * h[2]])


def lattice_index(box: BoxSpec, fine: bool) -> np.ndarray:
    shape = box.fine_shape if fine else box.coarse_shape
    k, j, i = np.meshgrid(np.arange(shape[2]), np.arange(shape[1]), np.arange(shape[0]),
                          indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()])


def boundary_mask(box: BoxSpec, fine: bool) -> np.ndarray:
    """True where a node lies on a Dirichlet face (lattice test only)."""
    idx = lattice_index(box, fine)
    shape = box.fine_shape if fine else box.coarse_shape
    m = np.zeros(idx.shape[1], dtype=bool)
    for a in range(3):
        if (box.periodic_mask >> a) & 1:
            continue
        if (box.dirichlet_mask >> (2 * a)) & 1:
            m |= idx[a] == 0
        if (box.dirichlet_mask >> (2 * a + 1)) & 1:
            m |= idx[a] == shape[a] - 1
    return m


# ------------------------------------------------------------ random fields --

def fourier_modes(rng: np.random.Generator, nmodes: int = 4, kmax: int = 3):
    """Random divergence-free Fourier modes: wave vectors in {-kmax..kmax}^3 \\ 0,
    phases in [0, 2 pi), unit amplitudes perpendicular to the wave vector."""
    modes = []
    while len(modes) < nmodes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if not np.any(k):
            continue
        phase = rng.uniform(0.0, 2.0 * np.pi)
        a = rng.standard_normal(3)
        a -= a.dot(k) / k.dot(k) * k
        a /= np.linalg.norm(a)
        modes.append((k.astype(np.float64), phase, a))
    return modes


def fourier_velocity(modes, pts: np.ndarray, box_len) -> np.ndarray:
    """Sum of the modes sampled at points [3][N] of a box with period box_len."""
    s = pts / np.asarray(box_len, dtype=np.float64)[:, None]
    out = np.zeros_like(pts)
    for k, phase, a in modes:
        arg = 2.0 * np.pi * (k @ s) + phase
        out += a[:, None] * np.sin(arg)[None, :]
    return out


def channel_profile(y: np.ndarray, z: np.ndarray, H: float = 0.41, U: float = U_MAX) -> np.ndarray:
    """Parabolic inflow profile with peak U at the channel centre."""
    return 16.0 * U * y * z * (H - y) * (H - z) / H ** 4


@dataclasses.dataclass
class StepInputs:
    """Inputs of one correction step: coarse solution x^L [4][N_c] (u, v, w, p),
    previous fine velocity v_prev [3][N_f], forcing mid-values (None = 0)."""
    xc: np.ndarray
    vprev: np.ndarray
    fmid: np.ndarray | None = None


def step_inputs(w: Workload, seed: int = 0) -> StepInputs:
    rng = np.random.default_rng(seed)
    box = w.box
    pc = node_coords(box, fine=False)
    pf = node_coords(box, fine=True)
    if w.kind == "fourier":
        modes = fourier_modes(rng)
        xc = np.zeros((4, box.n_coarse))
        xc[:3] = fourier_velocity(modes, pc, box.len)
        vprev = fourier_velocity(modes, pf, box.len)
        return StepInputs(xc, vprev)
    # channel: inflow profile extended in x plus 5 % noise on free nodes,
    # pressure a linear ramp towards the outflow plus noise
    sigma = 0.05 * U_MAX
    xc = np.zeros((4, box.n_coarse))
    xc[0] = channel_profile(pc[1], pc[2], box.len[1])
    free_c = ~boundary_mask(box, fine=False)
    xc[:3, free_c] += sigma * rng.standard_normal((3, int(free_c.sum())))
    walls_c = boundary_mask(box, fine=False) & (lattice_index(box, False)[0] > 0)
    xc[:3, walls_c] = 0.0
    xc[3] = 0.4 * (box.len[0] - pc[0]) + 0.05 * rng.standard_normal(box.n_coarse)
    vprev = np.zeros((3, box.n_fine))
    vprev[0] = channel_profile(pf[1], pf[2], box.len[1])
    free_f = ~boundary_mask(box, fine=True)
    vprev[:, free_f] += sigma * rng.standard_normal((3, int(free_f.sum())))
    walls_f = boundary_mask(box, fine=True) & (lattice_index(box, True)[0] > 0)
    vprev[:, walls_f] = 0.0
    return StepInputs(xc, vprev)


def mlp_params(nin: int, hidden: int, nout: int, seed: int = 0, bias_scale: float = 0.0):
    """Weights [fan_in][fan_out] ~ N(0, 1/fan_in); biases zero unless bias_scale > 0."""
    rng = np.random.default_rng(seed)
    dims = [(nin, hidden), (hidden, hidden), (hidden, nout)]
    out = []
    for fi, fo in dims:
        W = rng.standard_normal((fi, fo)) / np.sqrt(fi)
        b = bias_scale * rng.standard_normal(fo)
        out += [W, b]
    return out


def random_fine_field(box: BoxSpec, ncomp: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((ncomp, box.n_fine))


def random_coarse_field(box: BoxSpec, ncomp: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((ncomp, box.n_coarse))


def channel_initial(box: BoxSpec, amp: float = 0.3, seed: int = 0):
    """Divergence-free initial channel velocity at fine and coarse nodes: the
    inflow profile plus the curl of psi_z = a sin^2(pi x / L) s(y) s(z),
    s(t) = sin^2(pi t / H), which vanishes with its gradient on the inflow
    face and the walls.  Returns (fine [3][N_f], coarse [3][N_c])."""
    rng = np.random.default_rng(seed)
    a = amp * (1.0 + 0.2 * rng.standard_normal())
    Lx, H = box.len[0], box.len[1]
    out = []
    for fine in (True, False):
        p = node_coords(box, fine)
        x, y, z = p
        sx = np.sin(np.pi * x / Lx) ** 2
        sy, sz = np.sin(np.pi * y / H) ** 2, np.sin(np.pi * z / box.len[2]) ** 2
        dsy = 2 * np.sin(np.pi * y / H) * np.cos(np.pi * y / H) * np.pi / H
        dsx = 2 * np.sin(np.pi * x / Lx) * np.cos(np.pi * x / Lx) * np.pi / Lx
        v = np.zeros_like(p)
        v[0] = channel_profile(y, z, H) + a * sx * dsy * sz
        v[1] = -a * dsx * sy * sz
        out.append(v)
    return out[0], out[1]


def channel_dirichlet(box: BoxSpec, fine: bool):
    """(mask [4][N], values [4][N]) of the channel's Dirichlet velocity data:
    the inflow profile on x = 0, zero on the walls; pressure free."""
    p = node_coords(box, fine)
    m = boundary_mask(box, fine)
    mask = np.zeros((4, p.shape[1]), dtype=bool)
    mask[:3] = m[None, :]
    vals = np.zeros((4, p.shape[1]))
    inflow = m & (lattice_index(box, fine)[0] == 0)
    walls = m & ~inflow
    vals[0, inflow] = channel_profile(p[1, inflow], p[2, inflow], box.len[1])
    vals[:3, walls] = 0.0
    return mask, vals


# ------------------------------------------------- distorted hexahedral mesh --

def distorted_coords(box: BoxSpec, amp: float = 0.15, seed: int = 0, modes: int = 2) -> np.ndarray:
    """Fine node positions [3][N_f] of a smoothly distorted box (the synthetic
    stand-in for the paper's curved hexahedral meshes): the lattice positions
    plus, per component a, amp * H_a * sum_m s_m sin(pi k_a X_a / L_a)
    cos(2 pi k_b X_b / L_b + phi) cos(2 pi k_c X_c / L_c + psi), H_a the
    element size L_a / n_a, wavenumbers of about a quarter of the element
    count and random phases.  The displacement normal to each face vanishes
    on it, so the domain stays the box and boundary nodes slide along their
    faces.  Non-periodic boxes only."""
    if box.periodic_mask:
        raise ValueError("distorted meshes have no periodic axes")
    rng = np.random.default_rng(seed)
    P = node_coords(box, fine=True)
    H = [box.len[a] / box.n[a] for a in range(3)]
    out = P.copy()
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for _ in range(modes):
            ka = max(1, box.n[a] // 4) * int(rng.integers(1, 3))
            kb = int(rng.integers(0, max(1, box.n[b] // 4) + 1))
            kc = int(rng.integers(0, max(1, box.n[c] // 4) + 1))
            s = rng.uniform(0.5, 1.0) * (1 if rng.random() < 0.5 else -1) / modes
            phi, psi = rng.uniform(0, 2 * np.pi, 2)
            out[a] += (amp * H[a] * s * np.sin(np.pi * ka * P[a] / box.len[a])
                       * np.cos(2 * np.pi * kb * P[b] / box.len[b] + phi)
                       * np.cos(2 * np.pi * kc * P[c] / box.len[c] + psi))
    return out
