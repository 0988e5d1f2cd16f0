"""The paper's network form and inputs in plain FP64 numpy (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: only the tests, the smoke
check and the benchmark's CPU baseline may load it.

Network (arXiv 2307.14837, Sec. 3, layers f_1 .. f_L): no biases; batch
normalisation N_i(x) = (x - mu_i) / s_i * gamma_i + beta_i before each
activation (mu_i, s_i the mean and standard deviation estimated in
training); skip connections where input and output widths match:
    f_1(x) = tanh(N_1(W_1 x)),
    f_i(x) = tanh(N_i(W_i x)) + x,   i = 2 .. L - 1,
    f_L(x) = W_L x,
with L - 1 hidden layers of one width (8 in Sec. 5.3).  The activation is
tanh (the paper does not name it; the project's reading).

Inputs (Sec. 4.2): on each patch the prolongated velocities and pressure,
the nonlinear residual of all four equations, and 24 features of the coarse
cell's geometry: its 12 edge lengths, the 4 lengths of the diagonals between
vertices sharing no face, and for each of the 8 vertices the mean of the 3
angles between the faces meeting there.  Row layout (component-major):
[u, v, w, p at the patch nodes, r_u, r_v, r_w, r_p, edges (x-directed, then
y, then z), diagonals, vertex angles], 8 (2^J + 1)^3 + 24 values.
"""
from __future__ import annotations

import numpy as np

from . import _box, dofmap_levels, fine_nodes, level_box, patches

GEO_FEATURES = 24


def param_count(n_in, hidden, n_out, depth=8):
    """Trainable parameters: the weights of the depth + 1 layers and gamma,
    beta of the depth batch normalisations (the table of Sec. 5.3)."""
    return n_in * hidden + (depth - 1) * hidden * hidden + hidden * n_out + 2 * depth * hidden


def forward(X, Ws, gammas, betas, means, stds):
    """Y = f_L(... f_1(X)) row by row; Ws[i] is [fan_in][fan_out] (so W_i x is
    x @ Ws[i] for a row x); gammas .. stds hold one vector per hidden layer."""
    a = np.asarray(X, dtype=np.float64)
    depth = len(Ws) - 1
    for i in range(depth):
        z = a @ Ws[i]
        n = (z - means[i]) / stds[i] * gammas[i] + betas[i]
        h = np.tanh(n)
        a = h if i == 0 else h + a
    return a @ Ws[depth]


def _corners(box, I, J, K):
    """Coordinates [8][3] of the corners of coarse cell (I, J, K), vertex
    j = a + 2b + 4c at (I + a, J + b, K + c) times the cell sizes."""
    bx = _box(box)
    H = [bx.len[a] / bx.n[a] for a in range(3)]
    out = np.zeros((8, 3))
    for j in range(8):
        o = (j & 1, (j >> 1) & 1, j >> 2)
        out[j] = [(c + d) * h for c, d, h in zip((I, J, K), o, H)]
    return out


def geometry_features(P):
    """The 24 geometry features of a hexahedron with corners P [8][3] (vertex
    j = a + 2b + 4c): 12 edge lengths (edges along a, then b, then c, each
    ordered by the other two corner bits), 4 diagonal lengths (vertex j to its
    opposite 7 - j for j = 0, 1, 2, 3), and per vertex the mean of the three
    dihedral angles between the faces meeting at it."""
    P = np.asarray(P, dtype=np.float64)
    edges = []
    for axis in range(3):
        others = [a for a in range(3) if a != axis]
        for t in range(4):
            bits = [0, 0, 0]
            bits[others[0]] = t & 1
            bits[others[1]] = t >> 1
            j0 = bits[0] + 2 * bits[1] + 4 * bits[2]
            j1 = j0 + (1 << axis)
            edges.append(np.linalg.norm(P[j1] - P[j0]))
    diags = [np.linalg.norm(P[7 - j] - P[j]) for j in range(4)]
    angles = []
    for j in range(8):
        # the three edges leaving vertex j
        e = []
        for axis in range(3):
            k = j ^ (1 << axis)
            e.append(P[k] - P[j])
        # each face at j is spanned by two of the edges; the dihedral angle
        # along edge e_a is the angle between the faces (e_a, e_b) and
        # (e_a, e_c), measured in the plane normal to e_a
        ang = []
        for a in range(3):
            b, c = [x for x in range(3) if x != a]
            ea = e[a] / np.linalg.norm(e[a])
            pb = e[b] - ea * np.dot(e[b], ea)
            pc = e[c] - ea * np.dot(e[c], ea)
            cosv = np.dot(pb, pc) / (np.linalg.norm(pb) * np.linalg.norm(pc))
            ang.append(np.arccos(np.clip(cosv, -1.0, 1.0)))
        angles.append(np.mean(ang))
    return np.array(edges + diags + angles)


def paper_inputs(box, levels, x, r, shift=None, inv_scale=None):
    """Network inputs of the paper's form on the patches of the prediction
    `levels` (J) above the coarse mesh of `box`: [N_p, 8 (2^J + 1)^3 + 24],
    standardised as (X - shift) * inv_scale.  x, r [4][N_f] on the J-level
    lattice."""
    bx = _box(box)
    nf = fine_nodes(level_box(bx, levels))
    x = np.asarray(x, dtype=np.float64).reshape(4, nf)
    r = np.asarray(r, dtype=np.float64).reshape(4, nf)
    m, _ = dofmap_levels(bx, levels)
    nl = m.shape[1]
    npch = patches(bx)
    out = np.zeros((npch, 8 * nl + GEO_FEATURES))
    for c in range(4):
        out[:, nl * c:nl * (c + 1)] = x[c][m]
        out[:, 4 * nl + nl * c:4 * nl + nl * (c + 1)] = r[c][m]
    for M in range(npch):
        I = M % bx.n[0]
        J = (M // bx.n[0]) % bx.n[1]
        K = M // (bx.n[0] * bx.n[1])
        out[M, 8 * nl:] = geometry_features(_corners(bx, I, J, K))
    if shift is not None:
        out = out - np.asarray(shift, dtype=np.float64)
    if inv_scale is not None:
        out = out * np.asarray(inv_scale, dtype=np.float64)
    return out


def random_params(n_in, hidden, n_out, depth=8, seed=0):
    """Seeded parameters of the paper's network: weights N(0, 1/fan_in),
    gamma, beta, and the batch statistics mu, s of a trained state (seeded
    draws; s > 0)."""
    rng = np.random.default_rng(seed)
    dims = [n_in] + [hidden] * depth + [n_out]
    Ws = [rng.standard_normal((dims[i], dims[i + 1])) / np.sqrt(dims[i]) for i in range(depth + 1)]
    gammas = [1.0 + 0.2 * rng.standard_normal(hidden) for _ in range(depth)]
    betas = [0.1 * rng.standard_normal(hidden) for _ in range(depth)]
    means = [0.1 * rng.standard_normal(hidden) for _ in range(depth)]
    stds = [np.exp(0.3 * rng.standard_normal(hidden)) for _ in range(depth)]
    return Ws, gammas, betas, means, stds
