"""Closed forms printed in the paper (fixtures under tests/golden/)."""
import json
import os

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def test_network_parameter_counts():
    """8 hidden layers of equal width without biases, each with a BatchNorm
    scale and shift: N_in H + 7 H^2 + H N_out + 2 * 8 H (Sec. 3 and 5.3)."""
    g = json.load(open(GOLD))
    L = g["hidden_layers"]
    for row in g["network_sizes"]:
        H = row["hidden"]
        count = row["n_in"] * H + (L - 1) * H * H + H * row["n_out"] + 2 * L * H
        assert count == row["params"], row


def test_patch_dof_counts_and_samples():
    g = json.load(open(GOLD))
    d = 3
    assert (d + 1) * 3 ** d == g["patch_dofs_3d"]["J1"]
    assert (d + 1) * 5 ** d == g["patch_dofs_3d"]["J2"]
    # network output = velocity dofs of a patch; input = 2 * patch dofs + 24 geometry features
    assert d * 3 ** d == 81 and 2 * (d + 1) * 3 ** d + 24 == 240
    assert d * 5 ** d == 375
    assert g["patches"] * g["train_steps"] == g["train_samples"]
