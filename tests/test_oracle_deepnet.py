"""Pins of the oracle's form of the paper's network and inputs (Sec. 3 layers
with batch normalisation and skip connections; Sec. 4.2 inputs with 24
geometry features; Sec. 5.3 parameter table)."""
import json
import os

import numpy as np
import pytest
import torch

import dnnmg_synth as syn

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


@pytest.fixture(scope="module")
def dn(orc):
    from oracle import deepnet

    return deepnet


def test_parameter_table(dn):
    """The constructed network's parameter arrays hold exactly the trainable
    parameter counts of the Sec. 5.3 table (weights without biases, gamma and
    beta of each batch normalisation; mu and s are statistics)."""
    g = json.load(open(GOLD))
    for row in g["network_sizes"]:
        Ws, ga, be, mu, sd = dn.random_params(row["n_in"], 16, row["n_out"], g["hidden_layers"], seed=0)
        assert len(Ws) == g["hidden_layers"] + 1
        assert dn.param_count(row["n_in"], row["hidden"], row["n_out"], g["hidden_layers"]) == row["params"]
        small = sum(w.size for w in Ws) + sum(x.size for x in ga) + sum(x.size for x in be)
        assert small == dn.param_count(row["n_in"], 16, row["n_out"], g["hidden_layers"])


def torch_reference(X, Ws, ga, be, mu, sd):
    """The same network assembled from torch.nn modules (FP64, eval mode):
    Linear without bias, BatchNorm1d with the given statistics, Tanh,
    and the skip connections."""
    depth = len(Ws) - 1
    lin = [torch.nn.Linear(w.shape[0], w.shape[1], bias=False).double() for w in Ws]
    # eps below the rounding of s^2 (torch needs a positive one)
    bns = [torch.nn.BatchNorm1d(w.shape[1], eps=1e-30).double() for w in Ws[:-1]]
    with torch.no_grad():
        for l, w in zip(lin, Ws):
            l.weight.copy_(torch.as_tensor(w.T))
        for i, b in enumerate(bns):
            b.weight.copy_(torch.as_tensor(ga[i]))
            b.bias.copy_(torch.as_tensor(be[i]))
            b.running_mean.copy_(torch.as_tensor(mu[i]))
            b.running_var.copy_(torch.as_tensor(sd[i] ** 2))
            b.eval()
        a = torch.as_tensor(X)
        for i in range(depth):
            h = torch.tanh(bns[i](lin[i](a)))
            a = h if i == 0 else h + a
        return lin[depth](a).numpy()


@pytest.mark.parametrize("n_in,H,n_out,depth", [(240, 32, 81, 8), (1024, 24, 375, 8), (7, 5, 3, 3)])
def test_forward_matches_torch_modules(dn, n_in, H, n_out, depth):
    Ws, ga, be, mu, sd = dn.random_params(n_in, H, n_out, depth, seed=1)
    X = np.random.default_rng(2).standard_normal((37, n_in))
    got = dn.forward(X, Ws, ga, be, mu, sd)
    want = torch_reference(X, Ws, ga, be, mu, sd)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_skip_connections_carry_the_first_layer(dn):
    """With zero weights in layers 2 .. L-1 and beta = gamma mu / s (so the
    normalised zero is zero), every hidden layer passes its input on: the
    output is W_L f_1(x).  A missing skip gives zero instead."""
    Ws, ga, be, mu, sd = dn.random_params(9, 6, 4, 5, seed=3)
    for i in range(1, 5):
        Ws[i] = np.zeros_like(Ws[i])
        be[i] = ga[i] * mu[i] / sd[i]
    X = np.random.default_rng(4).standard_normal((11, 9))
    a1 = np.tanh((X @ Ws[0] - mu[0]) / sd[0] * ga[0] + be[0])
    assert np.allclose(dn.forward(X, Ws, ga, be, mu, sd), a1 @ Ws[5], rtol=1e-14, atol=1e-14)


def test_geometry_features_closed_forms(dn):
    H = np.array([0.3, 0.7, 1.1])
    P = np.array([[(j & 1) * H[0], ((j >> 1) & 1) * H[1], (j >> 2) * H[2]] for j in range(8)])
    f = dn.geometry_features(P)
    assert np.allclose(f[:12], np.repeat(H, 4), rtol=1e-15)
    assert np.allclose(f[12:16], np.sqrt(np.sum(H * H)), rtol=1e-15)
    assert np.allclose(f[16:], np.pi / 2, rtol=1e-15)
    # invariance under a rotation and a translation
    q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((3, 3)))
    assert np.allclose(dn.geometry_features(P @ q.T + 0.4), f, rtol=1e-12)
    # parallelepiped spanned by e1, e2 = (cos t, sin t, 0), e3: at vertex 0
    # the dihedral angles are t (along e3) and pi/2 twice; over all vertices
    # the mean of the vertex means is pi/2
    t = 1.1
    e = [np.array([1.0, 0, 0]), np.array([np.cos(t), np.sin(t), 0.0]), np.array([0, 0, 1.0])]
    P2 = np.array([(j & 1) * e[0] + ((j >> 1) & 1) * e[1] + (j >> 2) * e[2] for j in range(8)])
    g = dn.geometry_features(P2)
    assert abs(g[16] - (t + np.pi) / 3) <= 1e-14
    assert abs(np.mean(g[16:]) - np.pi / 2) <= 1e-14


@pytest.mark.parametrize("levels", [1, 2])
def test_paper_inputs_layout(orc, dn, levels):
    box = syn.channel_box((3, 2, 2))
    fb = orc.level_box(box, levels)
    nf = orc.fine_nodes(fb)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((4, nf))
    r = rng.standard_normal((4, nf))
    X = dn.paper_inputs(box, levels, x, r)
    nl = ((1 << levels) + 1) ** 3
    assert X.shape == (box.n_patches, 8 * nl + 24)
    assert X.shape[1] == (240 if levels == 1 else 1024)  # the table's N_in
    m, _ = orc.dofmap_levels(box, levels)
    M = 5
    for c in range(4):
        assert np.array_equal(X[M, nl * c:nl * (c + 1)], x[c, m[M]])
        assert np.array_equal(X[M, 4 * nl + nl * c:4 * nl + nl * (c + 1)], r[c, m[M]])
    H = np.array([box.len[a] / box.n[a] for a in range(3)])
    assert np.allclose(X[:, 8 * nl:8 * nl + 12], np.repeat(H, 4), rtol=1e-15)
    sh, inv = rng.standard_normal(X.shape[1]), rng.uniform(0.5, 2, X.shape[1])
    assert np.allclose(dn.paper_inputs(box, levels, x, r, sh, inv), (X - sh) * inv, rtol=1e-15, atol=1e-15)
