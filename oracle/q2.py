"""Plain FP64 CPU oracle of the DNN-MG fine level with the paper's Q2/Q2
elements on isoparametric hexahedra (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg load this module; the product path never does.  It shares no
code with the GPU library.  The arithmetic lives in ``q2_oracle.c`` (plain C,
no fast-math); this file marshals numpy arrays through ctypes and composes
the correction step from the oracle's own functions.

Every function cites the passage of arXiv 2307.14837 it follows:
  * ``apply``/``residual_b``/``rhs``  Sec. 2.2 eq. (disc:ns) with Q2/Q2 and
    pi_h: Q2 -> Q1; Sec. 2.3 eq. (4cranknicholson3) and (stabparams)
  * ``prolong``/``restrict``          Algorithm 1, transfer between the Q2
    spaces of levels L and L + 1
  * ``gather``/``features``           Sec. 4.2, eq. (defQ), network inputs
  * ``correction_step``               Algorithm 1 after the coarse solve
The element map is the Q2 interpolation of each element's 27 node positions;
the box topology is that of the Q1 library (n elements per axis = patches,
2n + 1 nodes per axis), with no periodic axes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import Box, NS, _box, _ns, _dp, _f64, mlp_forward_rows, norm2, eta_of, scatter

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "q2_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libq2oracle.so")

N_IN = 165
N_OUT = 81


def build(force: bool = True) -> str:
    """Compile the Q2 oracle with gcc (no fast-math); returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load(_LIB_PATH)
    return _lib


def load(path):
    """Open a compiled Q2 oracle (the tests also load altered copies)."""
    L = ctypes.CDLL(path)
    for f in ("q2_fine_nodes", "q2_coarse_nodes", "q2_elements"):
        getattr(L, f).restype = ctypes.c_int64
    L.q2_min_det.restype = ctypes.c_double
    return L


def _check(box):
    bx = _box(box)
    if bx.periodic_mask:
        raise ValueError("the Q2 mesh has no periodic axes")
    return bx


def fine_nodes(box) -> int:
    return int(lib().q2_fine_nodes(ctypes.byref(_box(box))))


def coarse_nodes(box) -> int:
    return int(lib().q2_coarse_nodes(ctypes.byref(_box(box))))


def elements(box) -> int:
    return int(lib().q2_elements(ctypes.byref(_box(box))))


def min_det(box, X) -> float:
    """Smallest Jacobian determinant of the element maps over the Gauss points."""
    bx = _check(box)
    X = _f64(X).reshape(3, fine_nodes(bx))
    return float(lib().q2_min_det(ctypes.byref(bx), _dp(X)))


def apply(box, ns, X, x, L=None) -> np.ndarray:
    """A(x) [4][N]: the iterate's terms of eq. (4cranknicholson3) with the
    LPS terms of eq. (disc:ns); X node positions [3][N]."""
    L = L or lib()
    bx = _check(box)
    nn = fine_nodes(bx)
    X = _f64(X).reshape(3, nn)
    x = _f64(x).reshape(4, nn)
    out = np.zeros((4, nn))
    L.q2_apply(ctypes.byref(bx), ctypes.byref(_ns(ns)), _dp(X), _dp(x), _dp(out))
    return out


def residual_b(box, ns, X, x, b, L=None) -> np.ndarray:
    """r = b - A(x), Dirichlet velocity rows 0 (Algorithm 1, fine residual)."""
    L = L or lib()
    bx = _check(box)
    nn = fine_nodes(bx)
    X = _f64(X).reshape(3, nn)
    x = _f64(x).reshape(4, nn)
    b = _f64(b).reshape(4, nn)
    out = np.zeros((4, nn))
    L.q2_residual_b(ctypes.byref(bx), ctypes.byref(_ns(ns)), _dp(X), _dp(x), _dp(b), _dp(out))
    return out


def rhs(box, ns, X, v, fmid=None, L=None) -> np.ndarray:
    """Right-hand side of eq. (4cranknicholson3) from velocity v [3][N]."""
    L = L or lib()
    bx = _check(box)
    nn = fine_nodes(bx)
    X = _f64(X).reshape(3, nn)
    v = _f64(v).reshape(3, nn)
    fmid = None if fmid is None else _f64(fmid).reshape(3, nn)
    out = np.zeros((4, nn))
    L.q2_rhs(ctypes.byref(bx), ctypes.byref(_ns(ns)), _dp(X), _dp(v), _dp(fmid), _dp(out))
    return out


def residual(box, ns, X, x, vprev, fmid=None, L=None) -> np.ndarray:
    """r = Rhs(vprev, fmid) - A(x): the residual of eq. (4cranknicholson3)."""
    return residual_b(box, ns, X, x, rhs(box, ns, X, vprev, fmid, L=L), L=L)


def prolong(box, xc) -> np.ndarray:
    """Q2 interpolation of [ncomp][N_c] coarse nodal values (coarse elements of
    2 x 2 x 2 fine elements) onto the fine nodes (Algorithm 1)."""
    bx = _check(box)
    if any(bx.n[a] % 2 for a in range(3)):
        raise ValueError("the coarse Q2 mesh needs an even element count per axis")
    xc = _f64(xc).reshape(-1, coarse_nodes(bx))
    out = np.zeros((xc.shape[0], fine_nodes(bx)))
    lib().q2_prolong(ctypes.byref(bx), ctypes.c_int(xc.shape[0]), _dp(xc), _dp(out))
    return out


def restrict(box, bf) -> np.ndarray:
    """Transpose of ``prolong`` on a fine dual vector [ncomp][N] (Algorithm 1)."""
    bx = _check(box)
    if any(bx.n[a] % 2 for a in range(3)):
        raise ValueError("the coarse Q2 mesh needs an even element count per axis")
    bf = _f64(bf).reshape(-1, fine_nodes(bx))
    out = np.zeros((bf.shape[0], coarse_nodes(bx)))
    lib().q2_restrict(ctypes.byref(bx), ctypes.c_int(bf.shape[0]), _dp(bf), _dp(out))
    return out


def features(box, X) -> np.ndarray:
    """Geometry inputs per element [N_e][3]: mean vertex-to-vertex edge length
    along each logical axis (Sec. 4.2 geometry inputs, read for curved cells)."""
    bx = _check(box)
    X = _f64(X).reshape(3, fine_nodes(bx))
    out = np.zeros((elements(bx), 3))
    lib().q2_features(ctypes.byref(bx), _dp(X), _dp(out))
    return out


def gather(box, X, x, r, shift=None, inv_scale=None) -> np.ndarray:
    """Network input batch [N_e][165] (eq. (defQ) on the fine Q2 elements plus
    the geometry inputs), standardised by shift / inv_scale."""
    bx = _check(box)
    nn = fine_nodes(bx)
    X = _f64(X).reshape(3, nn)
    x = _f64(x).reshape(-1, nn)
    r = _f64(r).reshape(-1, nn)
    out = np.zeros((elements(bx), N_IN))
    lib().q2_gather(ctypes.byref(bx), _dp(X), _dp(x), _dp(r), _dp(_f64(shift)),
                    _dp(_f64(inv_scale)), _dp(out))
    return out


def paper_inputs(box, X, x, r, shift=None, inv_scale=None):
    """Inputs of the paper's network (Sec. 4.2) on the fine Q2 elements:
    row M = [u, v, w, p at the 27 nodes, r_u, r_v, r_w, r_p there, the 24
    geometry features of the element's 8 vertices (general form)],
    standardised by shift / inv_scale.  x, r [4][N]."""
    from .deepnet import geometry_features

    bx = _check(box)
    nn = fine_nodes(bx)
    X = _f64(X).reshape(3, nn)
    x = _f64(x).reshape(4, nn)
    r = _f64(r).reshape(4, nn)
    nx, ny = 2 * bx.n[0] + 1, 2 * bx.n[1] + 1
    ne = elements(bx)
    out = np.zeros((ne, 8 * 27 + 24))
    for K in range(bx.n[2]):
        for J in range(bx.n[1]):
            for I in range(bx.n[0]):
                M = I + bx.n[0] * (J + bx.n[1] * K)
                nodes = [(2 * I + a) + nx * ((2 * J + b) + ny * (2 * K + c))
                         for c in range(3) for b in range(3) for a in range(3)]
                verts = [(2 * I + 2 * (j & 1)) + nx * ((2 * J + 2 * ((j >> 1) & 1)) + ny * (2 * K + 2 * (j >> 2)))
                         for j in range(8)]
                for c in range(4):
                    out[M, 27 * c:27 * (c + 1)] = x[c, nodes]
                    out[M, 108 + 27 * c:108 + 27 * (c + 1)] = r[c, nodes]
                out[M, 216:] = geometry_features(X[:, verts].T)
    if shift is not None:
        out -= np.asarray(shift, np.float64)
    if inv_scale is not None:
        out *= np.asarray(inv_scale, np.float64)
    return out


def correction_step(box, ns, X, params, xc, b, shift=None, inv_scale=None, indicator=False, threads=1,
                    network="mlp"):
    """Algorithm 1 after the coarse solve on the Q2 levels, in FP64:
    x~ = P x^L; r = b - A(x~); X = Q(x~, r, geometry); Y = N(X);
    x_corr = (v~ + L(Y), p~); b' = Rhs(v_corr); b'^L = R b'.
    b is the right-hand side of this step (the previous step's Rhs output).
    With indicator, also r(x_corr) and eta = ||r(x_corr)|| / ||r(x~)||."""
    xt = prolong(box, xc)
    r = residual_b(box, ns, X, xt, b)
    if network == "paper":
        from .deepnet import forward as deep_forward

        Xin = paper_inputs(box, X, xt, r, shift, inv_scale)
        Y = deep_forward(Xin, *params)
    else:
        Xin = gather(box, X, xt, r, shift, inv_scale)
        Y = mlp_forward_rows(Xin, params, threads)
    d = scatter(box, Y)
    vcorr = xt[:3] + d
    out = dict(xt=xt, r=r, X=Xin, Y=Y, d=d)
    if indicator:
        r2 = residual_b(box, ns, X, np.concatenate([vcorr, xt[3:4]]), b)
        out["r2"] = r2
        out["eta"] = eta_of(norm2(r), norm2(r2))
    bn = rhs(box, ns, X, vcorr)
    out.update(vcorr=vcorr, b=bn, bc=restrict(box, bn))
    return out
