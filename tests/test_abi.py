"""C-ABI library: loads, exports every declared symbol, validates on the host.

No call here reaches the GPU: only size queries and argument errors that the
library reports before anything is enqueued.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dnnmg.h")
LIB = os.path.join(ROOT, "paper_2307_14837_amd", "libdnnmg.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dnnmg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdnnmg.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    import paper_2307_14837_amd as L

    for n in declared():
        assert hasattr(L._lib.lib(), n)


def test_host_validation_without_gpu():
    import dnnmg_synth as syn
    import paper_2307_14837_amd as L

    box = L.Box.of(syn.cfg2().box)
    assert L.box_sizes(box) == (140481, 18785, 16384)
    # LPS corner sums (32 floats per patch), then one int per residual tile of
    # 16 x 8 x 4 nodes (9 x 5 x 9 tiles for 129 x 33 x 33 nodes), 256-byte blocks
    assert L.residual_workspace_bytes(box) == 16384 * 32 * 4 + 1792
    assert L.packed_bytes(L.BF16, 256, 0) == 192 * 256 * 2
    assert L.packed_bytes(L.FP8_E4M3, 512, 1) == 512 * 512  # E4M3 hidden product
    assert L.packed_bytes(L.FP8_E4M3, 512, 2) == 512 * 96 * 2  # BF16 output layer
    lib = L._lib.lib()
    # odd periodic axis is rejected before any launch
    bad = L.Box.of(syn.BoxSpec((3, 4, 4), (1, 1, 1), 7, 0))
    rc = lib.dnnmg_prolong(ctypes.byref(bad), 4, None, None, None)
    assert rc == -2 and b"even" in lib.dnnmg_last_error()
    rc = lib.dnnmg_prolong(ctypes.byref(box), 4, None, None, None)
    assert rc == -1
    rc = lib.dnnmg_prolong(ctypes.byref(box), 5, None, None, None)
    assert rc == -1
    net = L.MLP()
    net.n_in, net.hidden, net.n_out, net.dtype = 165, 100, 81, L.BF16
    rc = lib.dnnmg_patch_forward(ctypes.byref(net), 10, None, 192, None, None, None)
    assert rc == -3
    assert lib.dnnmg_version() >= 1


def test_graph_calls_validate_on_host():
    import paper_2307_14837_amd as L

    lib = L._lib.lib()
    # the legacy default stream cannot be captured; NULL handles are errors
    assert lib.dnnmg_graph_capture_begin(None) == -1
    assert lib.dnnmg_graph_replay(None, None) == -1
    assert lib.dnnmg_graph_destroy(None) == 0


def test_coarse_step_host_logic():
    """Levels and workspace of the GPU coarse solve are host computations:
    the meshes are the coarse mesh and its halvings while every axis keeps
    an even cell count; invalid options fail before any launch."""
    import dnnmg_synth as syn
    import paper_2307_14837_amd as L

    lib = L._lib.lib()
    o = L.coarse_opts(levels=0)  # every mesh of the hierarchy
    big = syn.cfg5().box  # coarse mesh 128 x 32 x 32 cells
    assert L.coarse_levels(big, o) == 4  # down to 16 x 4 x 4
    assert L.coarse_levels(big, L.coarse_opts(levels=3)) == 3
    assert L.coarse_levels(big, L.coarse_opts()) == 1  # the default: one mesh
    assert L.coarse_levels(syn.channel_box((16, 8, 8)), o) == 2
    # 6 x 4 x 4: the 3 x 2 x 2 mesh is not a level
    assert L.coarse_levels(syn.channel_box((6, 4, 4)), o) == 1
    # a periodic axis keeps an even cell count of at least 2 per box
    per = syn.BoxSpec((8, 8, 8), (1, 1, 1), 7, 0)
    assert L.coarse_levels(per, o) == 2
    for bad in (L.coarse_opts(krylov_dim=0), L.coarse_opts(newton_its=0), L.coarse_opts(omega=2.0),
                L.coarse_opts(fd_eta=0.0), L.coarse_opts(pre_sweeps=0)):
        assert lib.dnnmg_coarse_levels(ctypes.byref(L.Box.of(big)), ctypes.byref(bad)) == -1
    odd = L.Box.of(syn.channel_box((8, 2, 4)))
    assert lib.dnnmg_coarse_levels(ctypes.byref(odd), ctypes.byref(o)) == -2
    assert lib.dnnmg_coarse_workspace(ctypes.byref(odd), ctypes.byref(o)) == 0
    # the workspace holds every level's vectors, the local Vanka inverses
    # (108 x 108 FP32 per patch of meshes 128, 64, 32, 16 x ...) and the
    # FGMRES basis
    ws = L.coarse_workspace_bytes(big, o)
    n0 = 4 * 129 * 33 * 33
    inv = 108 * 108 * 4 * (16384 + 2048 + 256 + 32)
    assert ws > inv + 4 * n0 * (7 + 5 + 2 * o.krylov_dim + 1)
    assert ws < inv + 4 * n0 * 60
    # NULL workspace is an error before any launch
    rc = lib.dnnmg_coarse_solve(ctypes.byref(L.Box.of(big)), ctypes.byref(L.NS.of(syn.cfg5().ns)), None, None,
                                ctypes.byref(o), None, None, 0, None)
    assert rc == -1


def test_q2_host_validation_without_gpu():
    """The Q2 entry points check the mesh, the parameters and the pointers
    before anything is enqueued."""
    import dnnmg_synth as syn
    import paper_2307_14837_amd as L

    lib = L._lib.lib()
    ns = L.NS.of(syn.cfg2().ns)
    per = L.Box.of(syn.BoxSpec((4, 4, 4), (1, 1, 1), 1, 0))
    rc = lib.dnnmg_q2_residual_b(ctypes.byref(per), ctypes.byref(ns), None, None, None, None, None, 0, None)
    assert rc == -2 and b"periodic" in lib.dnnmg_last_error()
    box = L.Box.of(syn.channel_box((5, 2, 2)))
    rc = lib.dnnmg_q2_residual_b(ctypes.byref(box), ctypes.byref(ns), None, None, None, None, None, 0, None)
    assert rc == -1 and b"NULL" in lib.dnnmg_last_error()
    bad = L.NS(1e-3, 0.0, 0.02, 0.1)
    rc = lib.dnnmg_q2_rhs(ctypes.byref(box), ctypes.byref(bad), None, None, None, None, None, 0, None)
    assert rc == -1 and b"dt" in lib.dnnmg_last_error()
    # 189 floats per element (4 + 3 equations) in groups of 8, rounded up to 256 bytes; too small a workspace is rejected
    assert L.q2_workspace_bytes(box) == (3 * 8 * 189 * 4 + 255) // 256 * 256
    p = ctypes.c_void_p(16)
    rc = lib.dnnmg_q2_residual_b(ctypes.byref(box), ctypes.byref(ns), p, p, p, ctypes.c_void_p(32), p, 100, None)
    assert rc == -1 and b"workspace" in lib.dnnmg_last_error()
    # the coarse Q2 mesh needs even element counts
    rc = lib.dnnmg_q2_prolong(ctypes.byref(box), 4, None, None, None)
    assert rc == -2 and b"even" in lib.dnnmg_last_error()
    even = L.Box.of(syn.channel_box((4, 2, 2)))
    assert lib.dnnmg_q2_restrict(ctypes.byref(even), 0, None, None, None) == -1
    assert lib.dnnmg_q2_prolong(ctypes.byref(even), 4, None, None, None) == -1
    assert lib.dnnmg_q2_patch_features(ctypes.byref(even), None, None, None) == -1
    assert lib.dnnmg_q2_patch_features(ctypes.byref(per), None, None, None) == -2
    p = ctypes.c_void_p(16)
    feat = L.Feat(None, None)
    rc = lib.dnnmg_patch_gather_geom(ctypes.byref(even), None, p, p, ctypes.byref(feat), L.F32, 1.0, p, 192, None)
    assert rc == -1 and b"geom" in lib.dnnmg_last_error()
    rc = lib.dnnmg_patch_gather_geom(ctypes.byref(even), p, p, p, ctypes.byref(feat), L.F32, 1.0, p, 100, None)
    assert rc == -2
    net = L.MLP()
    net.n_in, net.hidden, net.n_out, net.dtype = 165, 128, 81, L.BF16
    rc = lib.dnnmg_patch_gather_forward_geom(ctypes.byref(even), ctypes.byref(net), None, p, p, ctypes.byref(feat),
                                             p, None)
    assert rc < 0


def test_residual_rhs_b_host_validation_without_gpu():
    """The fused indicator residual + Rhs and the predicated Rhs reject NULL
    and aliased pointers and a short workspace before anything is enqueued."""
    import dnnmg_synth as syn
    import paper_2307_14837_amd as L

    lib = L._lib.lib()
    ns = L.NS.of(syn.cfg2().ns)
    box = L.Box.of(syn.channel_box((4, 2, 2)))
    f = lib.dnnmg_residual_rhs_b
    x, b, r, s, ws = (ctypes.c_void_p(a) for a in (16, 32, 48, 64, 80))
    big = L.residual_workspace_bytes(box)
    assert f(ctypes.byref(box), ctypes.byref(ns), None, b, r, s, ws, big, None) == -1
    assert b"NULL" in lib.dnnmg_last_error()
    assert f(ctypes.byref(box), ctypes.byref(ns), x, b, b, s, ws, big, None) == -1
    assert f(ctypes.byref(box), ctypes.byref(ns), x, x, r, s, ws, big, None) == -1
    assert b"alias" in lib.dnnmg_last_error()
    assert f(ctypes.byref(box), ctypes.byref(ns), x, b, r, b, ws, big, None) == -1
    assert b"b_save" in lib.dnnmg_last_error()
    assert f(ctypes.byref(box), ctypes.byref(ns), x, b, r, s, ws, big - 1, None) == -2
    assert b"workspace" in lib.dnnmg_last_error()
    bad = L.NS(1e-3, 0.0, 0.02, 0.1)
    assert f(ctypes.byref(box), ctypes.byref(bad), x, b, r, s, ws, big, None) == -1
    rc = lib.dnnmg_rhs_if(ctypes.byref(box), ctypes.byref(ns), x, None, b, None, None)
    assert rc == -1 and b"NULL" in lib.dnnmg_last_error()


def test_mse_grad_loss_host_validation_without_gpu():
    """The fused loss gradient checks its size, pointers and workspace before
    anything is enqueued."""
    import paper_2307_14837_amd as L

    lib = L._lib.lib()
    p = ctypes.c_void_p(16)
    assert lib.dnnmg_mse_grad_loss(-1, p, p, p, p, p, 1 << 20, None) == -2
    assert lib.dnnmg_mse_grad_loss(10, None, p, p, p, p, 1 << 20, None) == -1
    assert b"NULL" in lib.dnnmg_last_error()
    assert lib.dnnmg_mse_grad_loss(10, p, p, p, p, p, L.norm2_workspace_bytes() - 1, None) == -2
    assert b"workspace" in lib.dnnmg_last_error()
