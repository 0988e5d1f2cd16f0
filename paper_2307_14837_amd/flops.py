"""Algorithmic work per unit of the hot-path kernels (used for roofline figures).

Flops count FP32 (or FP64) arithmetic as issued by the algorithm as written
in the kernels: add/sub/mul/max = 1, fused multiply-add = 2, sqrt/div = 1.
Halo recomputation, padding and inactive lanes are not counted.
Bytes count each input array read once and each output written once.
"""

# ---- building blocks of the sum-factorised 2x2x2 Gauss quadrature ----------
LIN2 = 5                 # two Gauss-point values of a linear function: sub + 2 fma
EVAL_VAL = 12 * LIN2     # values at 8 Gauss points: 3 passes x 4 lines
EVAL_VG = 24 + 34 + 40 + 16  # values + 3 gradient components (x, y, z passes, 1/h scaling)
INTEGRATE = 76 + 56 + 36     # transpose to 8 vertex integrals of (F, Gx, Gy, Gz)
INTEGRATE_FLUX = 52 + 56 + 36  # transpose of (Gx, Gy, Gz) only
PI_VERTICES = 24         # patch-corner values -> the fine cell's vertex values
PI_TRANSPOSE = 36        # vertex integrals -> patch-corner integrals


INTEGRATE_VAL = 12 * LIN2  # transpose of F only


def residual_flops_per_cell(lps: bool = False) -> int:
    """Crank-Nicolson residual r = F - A(x) per fine cell (Q1, 2x2x2 Gauss).

    lps=False: the Galerkin terms plus the test that the cell's vertex values
    equal their patch interpolant, the work done on a prolongated iterate
    (where every local projection term is exactly zero).  lps=True adds the
    local projection terms of eq. (disc:ns) as the algorithm needs them
    (no recomputation counted)."""
    values = 7 * EVAL_VAL                          # x~, vp, p~ at the Gauss points
    test = 4 * PI_VERTICES                         # patch interpolant of (x~, p~)
    per_comp = (16                                 # (1/k)(vp_a - v_a)
                + EVAL_VG + 56                     # grad vp_a; -1/2 vp . grad vp_a
                + EVAL_VG + 56 + 8                 # grad v_a; -1/2 v . grad v_a; divergence
                + 48 + 8                           # -nu/2 grad(vp_a + v_a), + p d_a phi
                + INTEGRATE)                       # vertex integrals
    cont = 8 + INTEGRATE_VAL                       # -(div x~, xi)
    sums = 32 + 32                                 # quadrature weight, LDS sums
    total = values + test + 3 * per_comp + cont + sums
    if lps:
        stab = 47 + 9                              # |v|_inf over vertices, alpha_T, delta_T
        pi_vals = 3 * EVAL_VAL                     # pi x~ at the Gauss points
        per_lps = EVAL_VG + 128 + INTEGRATE_FLUX + PI_TRANSPOSE + 16  # delta term, own + corners
        cont_lps = 8 + EVAL_VG + 24 + INTEGRATE_FLUX + 8 + PI_TRANSPOSE + 16  # alpha term
        total += stab + pi_vals + 3 * per_lps + cont_lps + 4 * 8  # corner sums
    return total


PROLONG_PER_NODE = 3 * 4  # Q1 interpolation of 4 fields: 12 two-point means per 8 fine nodes, each 2 flops


def prolong_residual_flops_per_cell() -> int:
    """Prolongation fused with the residual, per fine cell (about one fine
    node per cell): the Galerkin terms without the interpolant test, since a
    prolongated iterate has no local projection terms."""
    return residual_flops_per_cell(lps=False) - 4 * PI_VERTICES + PROLONG_PER_NODE


def prolong_residual_b_flops_per_cell() -> int:
    """Prolongation fused with r = b - A(x~) against a given right-hand side,
    per fine cell: only the terms of the new iterate, plus b at the node."""
    values = 4 * EVAL_VAL                          # x~, p~ at the Gauss points
    per_comp = (8                                  # -(1/k) v_a
                + EVAL_VG + 56 + 8                 # grad v_a; -1/2 v . grad v_a; divergence
                + 24 + 8                           # -nu/2 grad v_a, + p d_a phi
                + INTEGRATE)                       # vertex integrals
    cont = 8 + INTEGRATE_VAL                       # -(div x~, xi)
    sums = 32 + 32 + 4                             # quadrature weight, LDS sums, + b
    return values + 3 * per_comp + cont + sums + PROLONG_PER_NODE


def rhs_flops_per_cell() -> int:
    """Right-hand side b = Rhs(v) per fine cell (no forcing)."""
    per_comp = EVAL_VG + 8 + 24 + 7 * 8 + INTEGRATE
    return 3 * EVAL_VAL + 3 * per_comp + 24 + 24


def mlp_flops_per_patch(hidden: int, n_in: int = 165, n_out: int = 81) -> int:
    """Useful multiply-add flops of the 165-H-H-81 network per patch."""
    return 2 * (n_in * hidden + hidden * hidden + hidden * n_out)


def mlp_issued_flops_per_patch(hidden: int) -> int:
    """Flops issued on the padded MFMA shapes (K 165 -> 192, N 81 -> 96)."""
    return 2 * (192 * hidden + hidden * hidden + hidden * 96)


# ---- bytes per fine node (FP32 fields, each read or written once) ----------
BYTES_PER_FINE_NODE = {
    "prolong": 4 * 4 + 4 * 8 / 8,        # write 4 FP32 fields; read 4 FP64 coarse fields (1/8 node)
    "residual": 4 * 4 + 3 * 4 + 4 * 4,   # read x (4), vp (3); write r (4)
    "rhs": 3 * 4 + 4 * 4,                # read v (3); write b (4)
    # read x (4), b (4); write r (4), the next b (4) and the saved b (4)
    "residual_rhs_b": 4 * 4 + 4 * 4 + 3 * 4 * 4,
    "scatter": 81 * 4 / 8 + 4 * 4 + 4 * 4,  # read Y (81 per patch), x~ (4); write x_corr (4)
    "restrict": 4 * 4 + 4 * 8 / 8,       # read b (4); write 4 FP64 coarse fields
}


def gather_bytes_per_patch(x_bytes: int, ldx: int = 192) -> float:
    """Read 6 fine fields at the patch's nodes (about 8 fine nodes own one patch),
    write one padded row of the network input."""
    return 8 * 6 * 4 + ldx * x_bytes


# ---- algorithmic counts per fine node used for the roofline figures --------
# Per-node estimates of the steps of the correction, lower than the itemised
# counts above (they leave out the sum-factorisation bookkeeping): the fine
# residual about 1.3 k flop at a prolongated iterate (Galerkin terms; its
# local projection terms vanish there) and 2.9 k with active LPS terms; the
# right-hand side about 1.2 k; the prolongation under 10.  A kernel that
# evaluates only part of a step (the forms against the carried right-hand
# side leave the previous velocity's terms to the Rhs of the previous step)
# is credited with the step's estimate times the share of the itemised count
# that it evaluates.
ALG_RESIDUAL_AT_PROLONGATION_PER_NODE = 1300
ALG_RESIDUAL_GENERAL_PER_NODE = 2900
ALG_RHS_PER_NODE = 1200
ALG_PROLONG_PER_NODE = 10


def _share_prolong_residual_b() -> float:
    return prolong_residual_b_flops_per_cell() / prolong_residual_flops_per_cell()


def _share_residual_b_general() -> float:
    full = residual_flops_per_cell(lps=True)
    return (full - rhs_flops_per_cell()) / full


ALG_PROLONG_RESIDUAL_B_PER_NODE = round(
    (ALG_PROLONG_PER_NODE + ALG_RESIDUAL_AT_PROLONGATION_PER_NODE) * _share_prolong_residual_b())
ALG_RESIDUAL_B_GENERAL_PER_NODE = round(ALG_RESIDUAL_GENERAL_PER_NODE * _share_residual_b_general())
# the indicator's residual and the next step's right-hand side at one iterate
ALG_RESIDUAL_RHS_B_GENERAL_PER_NODE = ALG_RESIDUAL_B_GENERAL_PER_NODE + ALG_RHS_PER_NODE


# ---- Q2/Q2 elements on curved hexahedra (27 Gauss points per element) -----
# Counted as the element kernel evaluates them, with sum factorisation: the
# node values go to the points by three 1-D passes of 3 terms, the weak-form
# coefficients back to the nodes likewise; the per-point work (Jacobian
# inverse, physical gradients, the 8 vertex Q1 interpolants, the 28
# coefficients) is counted once per point.


def q2_residual_flops_per_element() -> int:
    """r = b - A(x) on one Q2 element (momentum and continuity rows with both
    LPS terms), as issued by the element kernel."""
    interp = 7 * (27 * 2 * 6 + 27 * 3 * 6 + 27 * 4 * 6) - 3 * 27 * 6  # 7 quantities, coordinates without values
    pi_interp = 8 * (8 + 15 * 2)                  # Q1 functions of 8 vertices, pi v, grad pi v, grad pi p
    point = (14 + 9 * 3 + 1 + 3                   # det, inverse, weight
             + (9 + 9 + 3 + 3) * 5                # physical gradients of v, pi v, p, pi p
             + 3 * 5 + 3 * 6                      # convection, R_a
             + 3 * (15 + 6 + 4 + 30) + 30)        # momentum and continuity coefficients
    test = 4 * (27 * (12 + 6 + 6) + 27 * 6 + 27 * 6) + 4 * (18 * 12 + 12 * 9 + 8 * 6)  # x, y, z passes; vertices
    stab = 28 * 8 + 27 * 6 + 10                   # h_T, |v|_inf, alpha_T, delta_T
    return interp + 27 * (pi_interp + point) + test + stab


def q2_rhs_flops_per_element() -> int:
    """b = Rhs(v) on one Q2 element (momentum rows), as issued."""
    interp = 6 * (27 * 2 * 6 + 27 * 3 * 6 + 27 * 4 * 6) - 3 * 27 * 6 + 3 * 3 * 27 * 6
    point = 14 + 9 * 3 + 4 + 9 * 5 + 15 + 3 * (6 + 15)
    test = 3 * (27 * (12 + 6 + 6) + 27 * 6 + 27 * 6)
    return interp + 27 * point + test


def q2_sum_nodes_bytes_per_node() -> float:
    """Per-node sum of the element vectors: 108 floats per element read once
    (one element per 8 nodes of the lattice), b read and r written (4
    fields each)."""
    return 108 * 4 / 8 + 4 * 4 + 4 * 4


# r = b - A(x) on the Q2 mesh: x (4 FP32 fields) and b read, r written, the
# FP64 node positions read, once per node (the element vectors' round trip
# through the workspace is not counted)
Q2_RESIDUAL_BYTES_PER_NODE = 4 * 4 + 4 * 4 + 4 * 4 + 3 * 8
