"""Plain FP64 CPU oracle for the DNN-MG fine-level correction (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg load this module; the product path never does.  It shares no code
with the GPU library.  The arithmetic lives in ``dnnmg_oracle.c`` (plain C,
no fast-math); this file only marshals numpy arrays through ctypes.

Every function cites the passage of arXiv 2307.14837 it follows:
  * ``dofmap``              Sec. 4.2, dof map and valence vector mu
  * ``prolong``/``restrict`` Algorithm 1, prolongation and restriction of the rhs
  * ``residual``/``rhs``    Sec. 2.3, eq. (4cranknicholson3) with (stabparams)
                            and the LPS terms of eq. (disc:ns)
  * ``gather``              eqs. (Eq:DefR), (eq:defQ) and the network inputs
  * ``scatter``             eq. (defL)
  * ``mlp_forward``/``mlp_backward``/``adamw``  Sec. 3, Sec. 4.2 training
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dnnmg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

N_IN = 165
N_OUT = 81


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math); returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Box(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("len", ctypes.c_double * 3),
        ("periodic_mask", ctypes.c_uint32),
        ("dirichlet_mask", ctypes.c_uint32),
    ]


class NS(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("dt", ctypes.c_double),
                ("alpha0", ctypes.c_double), ("delta0", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load(_LIB_PATH)
    return _lib


def load(path):
    """Open a compiled oracle library and declare its signatures (the tests
    also load deliberately altered copies of the oracle this way)."""
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    d = ctypes.c_double
    i64 = ctypes.c_int64
    dp = P(d)
    L.or_fine_nodes.restype = i64
    L.or_coarse_nodes.restype = i64
    L.or_patches.restype = i64
    L.or_mse.restype = d
    L.or_norm2.restype = d
    L.or_round_bf16.restype = d
    L.or_round_bf16.argtypes = [d]
    L.or_round_e4m3.restype = d
    L.or_round_e4m3.argtypes = [d]
    L.or_mlp_forward.argtypes = [i64, ctypes.c_int, ctypes.c_int, ctypes.c_int] + [dp] * 10
    L.or_mlp_backward.argtypes = [i64, ctypes.c_int, ctypes.c_int, ctypes.c_int] + [dp] * 12
    L.or_mse.argtypes = [i64, ctypes.c_int, dp, dp, dp]
    L.or_adamw.argtypes = [i64, dp, dp, dp, dp, d, d, d, d, d, i64]
    L.or_norm2.argtypes = [i64, dp, dp]
    L.or_vanka_sweep.argtypes = [P(Box), P(NS), dp, dp, dp, d, ctypes.c_int, dp]
    return L


def _box(b) -> Box:
    """Accept an oracle Box or any object with n/len/periodic_mask/dirichlet_mask."""
    if isinstance(b, Box):
        return b
    bx = Box()
    for a in range(3):
        bx.n[a] = int(b.n[a])
        bx.len[a] = float(b.len[a])
    bx.periodic_mask = int(b.periodic_mask)
    bx.dirichlet_mask = int(b.dirichlet_mask)
    return bx


def _ns(p) -> NS:
    if isinstance(p, NS):
        return p
    return NS(float(p.nu), float(p.dt), float(p.alpha0), float(p.delta0))


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def fine_nodes(box) -> int:
    return int(lib().or_fine_nodes(ctypes.byref(_box(box))))


def coarse_nodes(box) -> int:
    return int(lib().or_coarse_nodes(ctypes.byref(_box(box))))


def patches(box) -> int:
    return int(lib().or_patches(ctypes.byref(_box(box))))


def dirichlet_flags(box) -> np.ndarray:
    out = np.zeros(fine_nodes(box), dtype=np.uint8)
    lib().or_dirichlet_flags(ctypes.byref(_box(box)), out.ctypes.data_as(ctypes.c_void_p))
    return out


def dofmap(box):
    """dof(P_M, iota) [N_p, 27] int32 and the valence count per fine node (Sec. 4.2)."""
    bx = _box(box)
    m = np.zeros((patches(bx), 27), dtype=np.int32)
    mult = np.zeros(fine_nodes(bx), dtype=np.uint8)
    lib().or_dofmap(ctypes.byref(bx), m.ctypes.data_as(ctypes.c_void_p),
                    mult.ctypes.data_as(ctypes.c_void_p))
    return m, mult


def prolong(box, xc) -> np.ndarray:
    """Q1 prolongation coarse -> fine of [ncomp][N_c] (Algorithm 1, prolongation)."""
    bx = _box(box)
    xc = _f64(xc).reshape(-1, coarse_nodes(bx))
    out = np.zeros((xc.shape[0], fine_nodes(bx)))
    lib().or_prolong(ctypes.byref(bx), ctypes.c_int(xc.shape[0]), _dp(xc), _dp(out))
    return out


def restrict(box, bf) -> np.ndarray:
    """Transpose of the prolongation applied to a fine dual vector (Algorithm 1, restriction)."""
    bx = _box(box)
    bf = _f64(bf).reshape(-1, fine_nodes(bx))
    out = np.zeros((bf.shape[0], coarse_nodes(bx)))
    lib().or_restrict(ctypes.byref(bx), ctypes.c_int(bf.shape[0]), _dp(bf), _dp(out))
    return out


def residual(box, ns, x, vprev, fmid=None) -> np.ndarray:
    """r = F - A(x) of eq. (4cranknicholson3); x [4][N_f], vprev [3][N_f], fmid [3][N_f]."""
    bx = _box(box)
    nf = fine_nodes(bx)
    x = _f64(x).reshape(4, nf)
    vprev = _f64(vprev).reshape(3, nf)
    fmid = None if fmid is None else _f64(fmid).reshape(3, nf)
    out = np.zeros((4, nf))
    lib().or_residual(ctypes.byref(bx), ctypes.byref(_ns(ns)), _dp(x), _dp(vprev), _dp(fmid), _dp(out))
    return out


def rhs(box, ns, v, fmid=None) -> np.ndarray:
    """Right-hand side of eq. (4cranknicholson3) built from velocity v [3][N_f]."""
    bx = _box(box)
    nf = fine_nodes(bx)
    v = _f64(v).reshape(3, nf)
    fmid = None if fmid is None else _f64(fmid).reshape(3, nf)
    out = np.zeros((4, nf))
    lib().or_rhs(ctypes.byref(bx), ctypes.byref(_ns(ns)), _dp(v), _dp(fmid), _dp(out))
    return out


def gather(box, x, r, shift=None, inv_scale=None) -> np.ndarray:
    """Network input batch [N_p, 165]: Q(v~), Q(r_mom), coarse cell sizes, standardised."""
    bx = _box(box)
    nf = fine_nodes(bx)
    x = _f64(x).reshape(-1, nf)
    r = _f64(r).reshape(-1, nf)
    out = np.zeros((patches(bx), N_IN))
    lib().or_gather(ctypes.byref(bx), _dp(x), _dp(r), _dp(_f64(shift)), _dp(_f64(inv_scale)), _dp(out))
    return out


def scatter(box, Y) -> np.ndarray:
    """Extension L of eq. (defL): multiplicity-averaged patch outputs [3][N_f]."""
    bx = _box(box)
    Y = _f64(Y).reshape(patches(bx), N_OUT)
    out = np.zeros((3, fine_nodes(bx)))
    lib().or_scatter(ctypes.byref(bx), _dp(Y), _dp(out))
    return out


# ------------------------------------------- J-level prediction (Sec. 4.2) --

def level_box(box, J) -> Box:
    """The box whose fine lattice is the prediction lattice J levels above the
    coarse mesh of `box` (n * 2^(J-1) cells per axis)."""
    bx = _box(box)
    out = Box()
    for a in range(3):
        out.n[a] = int(bx.n[a]) << (J - 1)
        out.len[a] = bx.len[a]
    out.periodic_mask, out.dirichlet_mask = bx.periodic_mask, bx.dirichlet_mask
    return out


def patch_nodes(J) -> int:
    return ((1 << J) + 1) ** 3


def dofmap_levels(box, J):
    """dof(P_M, iota) [N_p, (2^J+1)^3] and valence on the J-level lattice."""
    bx = _box(box)
    m = np.zeros((patches(bx), patch_nodes(J)), dtype=np.int32)
    mult = np.zeros(fine_nodes(level_box(bx, J)), dtype=np.uint8)
    lib().or_dofmap_levels(ctypes.byref(bx), ctypes.c_int(J), m.ctypes.data_as(ctypes.c_void_p),
                           mult.ctypes.data_as(ctypes.c_void_p))
    return m, mult


def prolong_levels(box, J, xc) -> np.ndarray:
    """P^J: the prolongation of Algorithm 1 applied J times (coarse mesh of
    `box` to the J-level lattice)."""
    x = _f64(xc)
    for lev in range(1, J + 1):
        x = prolong(level_box(box, lev), x)
    return x


def restrict_levels(box, J, bf) -> np.ndarray:
    """(P^J)^T: the restriction applied J times (J-level lattice to the coarse
    mesh of `box`)."""
    b = _f64(bf)
    for lev in range(J, 0, -1):
        b = restrict(level_box(box, lev), b)
    return b


def gather_levels(box, J, x, r, shift=None, inv_scale=None) -> np.ndarray:
    """Network input batch of the J-level prediction [N_p, 6 (2^J+1)^3 + 3]."""
    bx = _box(box)
    nf = fine_nodes(level_box(bx, J))
    x = _f64(x).reshape(-1, nf)
    r = _f64(r).reshape(-1, nf)
    out = np.zeros((patches(bx), 6 * patch_nodes(J) + 3))
    lib().or_gather_levels(ctypes.byref(bx), ctypes.c_int(J), _dp(x), _dp(r), _dp(_f64(shift)),
                           _dp(_f64(inv_scale)), _dp(out))
    return out


def scatter_levels(box, J, Y) -> np.ndarray:
    """Extension L of eq. (defL) on the J-level patches: [3][N_f]."""
    bx = _box(box)
    nf = fine_nodes(level_box(bx, J))
    Y = _f64(Y).reshape(patches(bx), 3 * patch_nodes(J))
    out = np.zeros((3, nf))
    lib().or_scatter_levels(ctypes.byref(bx), ctypes.c_int(J), _dp(Y), _dp(out))
    return out


def mlp_forward(X, W1, b1, W2, b2, W3, b3, want_hidden=False):
    """Y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3 per row (Sec. 3, tanh MLP)."""
    X = _f64(X)
    n, nin = X.shape
    H = W1.shape[1]
    nout = W3.shape[1]
    W1, W2, W3 = _f64(W1), _f64(W2), _f64(W3)
    b1, b2, b3 = _f64(b1), _f64(b2), _f64(b3)
    Y = np.zeros((n, nout))
    A1 = np.zeros((n, H)) if want_hidden else None
    A2 = np.zeros((n, H)) if want_hidden else None
    lib().or_mlp_forward(n, nin, H, nout, _dp(X), _dp(W1), _dp(b1), _dp(W2), _dp(b2), _dp(W3),
                         _dp(b3), _dp(Y), _dp(A1), _dp(A2))
    return (Y, A1, A2) if want_hidden else Y


def mlp_backward(X, W2, W3, A1, A2, dY):
    """Parameter gradients of sum <dY, Y> through the tanh MLP (chain rule)."""
    X, W2, W3, A1, A2, dY = map(_f64, (X, W2, W3, A1, A2, dY))
    n, nin = X.shape
    H = W2.shape[0]
    nout = W3.shape[1]
    dW1 = np.zeros((nin, H)); db1 = np.zeros(H)
    dW2 = np.zeros((H, H)); db2 = np.zeros(H)
    dW3 = np.zeros((H, nout)); db3 = np.zeros(nout)
    lib().or_mlp_backward(n, nin, H, nout, _dp(X), _dp(W2), _dp(W3), _dp(A1), _dp(A2), _dp(dY),
                          _dp(dW1), _dp(db1), _dp(dW2), _dp(db2), _dp(dW3), _dp(db3))
    return dW1, db1, dW2, db2, dW3, db3


def mse(Y, T):
    """Training loss (1/n) sum ||Y_M - T_M||^2 and dY (Sec. 4.2, training objective)."""
    Y, T = _f64(Y), _f64(T)
    dY = np.zeros_like(Y)
    loss = lib().or_mse(Y.shape[0], Y.shape[1], _dp(Y), _dp(T), _dp(dY))
    return float(loss), dY


def adamw(theta, m, v, g, lr, b1, b2, eps, wd, t):
    """One AdamW step in place (Sec. 3: AdamW optimiser)."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    g = _f64(g)
    lib().or_adamw(theta.size, _dp(theta), _dp(m), _dp(v), _dp(g), lr, b1, b2, eps, wd, int(t))


def norm2(a, b=None) -> float:
    a = _f64(a).ravel()
    b = None if b is None else _f64(b).ravel()
    return float(lib().or_norm2(a.size, _dp(a), _dp(b)))


def round_bf16(x) -> np.ndarray:
    f = lib().or_round_bf16
    return np.vectorize(lambda t: f(float(t)), otypes=[np.float64])(np.asarray(x, dtype=np.float64))


def round_e4m3(x) -> np.ndarray:
    f = lib().or_round_e4m3
    return np.vectorize(lambda t: f(float(t)), otypes=[np.float64])(np.asarray(x, dtype=np.float64))


def eta_of(n0, n1) -> float:
    """Indicator eta = ||r(x_corr)|| / ||r(x~)|| from the two squared norms;
    0/0 (both residuals zero) reads as 0, a zero reference with a nonzero
    corrected residual as +inf."""
    if n0 > 0.0:
        return float(np.sqrt(n1 / n0))
    return 0.0 if n1 == 0.0 else float("inf") if n1 > 0.0 else float("nan")


def fallback_taken(n0, n1, theta) -> int:
    """Fallback decision of the residual indicator: eta > theta or eta NaN,
    where theta = +inf disables the fallback."""
    if np.isinf(theta):
        return 0
    eta = eta_of(n0, n1)
    return int(not (eta <= theta))


def mlp_forward_rows(X, params, threads=1):
    """mlp_forward over row ranges on `threads` host threads (the network acts
    on each patch row alone, so every row's arithmetic is unchanged)."""
    if threads <= 1 or X.shape[0] < 2 * threads:
        return mlp_forward(X, *params)
    from concurrent.futures import ThreadPoolExecutor

    X = _f64(X)
    parts = np.array_split(np.arange(X.shape[0]), threads)
    with ThreadPoolExecutor(threads) as ex:
        Ys = list(ex.map(lambda idx: mlp_forward(X[idx[0]:idx[-1] + 1], *params), parts))
    return np.concatenate(Ys)


def correction_step(box, ns, params, xc, vprev, shift=None, inv_scale=None, indicator=False,
                    theta=1.0, fallback_sweeps=4, omega=1.0, threads=1, levels=1):
    """Algorithm 1 after the coarse solve, step by step in FP64:
    x~ = P x^L; r = F - A(x~); X = Q(x~, r, geometry); Y = N(X);
    x_corr = (v~ + L(Y), p~); b = Rhs(v~ + d); b^L = R b.
    With indicator, also r(x_corr) and eta = ||r(x_corr)|| / ||r(x~)||.
    threads > 1 evaluates the network's rows on that many host threads.
    levels = J: the prediction J levels above the coarse mesh (Sec. 4.2):
    P and R are applied J times, the residual, Rhs and fallback live on the
    J-level lattice (the fine mesh of level_box(box, J)), the patches are
    the coarse cells with (2^J + 1)^3 nodes."""
    if levels == 1:
        xt = prolong(box, xc)
    else:
        xt = prolong_levels(box, levels, xc)
        fine_box = level_box(box, levels)
        box, coarse_box = fine_box, box
    r = residual(box, ns, xt, vprev)
    if levels == 1:
        X = gather(box, xt, r, shift, inv_scale)
    else:
        X = gather_levels(coarse_box, levels, xt, r, shift, inv_scale)
    Y = mlp_forward_rows(X, params, threads)
    d = scatter(box, Y) if levels == 1 else scatter_levels(coarse_box, levels, Y)
    vcorr = xt[:3] + d
    out = dict(xt=xt, r=r, X=X, Y=Y, d=d)
    if indicator:
        # residual indicator; above theta the plain fine correction
        # (pressure-held patch sweeps from x~) replaces the network's
        xcorr = np.concatenate([vcorr, xt[3:4]])
        r2 = residual(box, ns, xcorr, vprev)
        out["r2"] = r2
        n0, n1 = norm2(r), norm2(r2)
        out["eta"] = eta_of(n0, n1)
        out["fell_back"] = fallback_taken(n0, n1, theta)
        if out["fell_back"]:
            xv = xt.copy()
            for _ in range(fallback_sweeps):
                xv = vanka_sweep(box, ns, xv, vprev, omega=omega, coupled=False)
            vcorr = xv[:3]
    b = rhs(box, ns, vcorr)
    bc = restrict(box, b) if levels == 1 else restrict_levels(coarse_box, levels, b)
    out.update(vcorr=vcorr, b=b, bc=bc)
    return out


def vanka_matrix(box, ns, w, M) -> np.ndarray:
    """Local 108 x 108 matrix of the plain fine-level correction on patch M
    (Picard linearisation at velocity w, the patch's own cells; see the C
    source for the blocks)."""
    bx = _box(box)
    w = _f64(w).reshape(-1, fine_nodes(bx))
    A = np.zeros((108, 108))
    lib().or_vanka_matrix(ctypes.byref(bx), ctypes.byref(_ns(ns)), _dp(w), ctypes.c_int64(M), _dp(A))
    return A


def dense_solve(A, b) -> np.ndarray:
    A = np.array(A, dtype=np.float64, order="C")
    x = np.array(b, dtype=np.float64)
    rc = lib().or_dense_solve(ctypes.c_int(A.shape[0]), _dp(A), _dp(x))
    if rc:
        raise np.linalg.LinAlgError("singular")
    return x


def vanka_sweep(box, ns, x, vprev, fmid=None, omega=1.0, coupled=False) -> np.ndarray:
    """One additive patch sweep with L-averaging: the plain fine-level
    correction used by the residual-indicator fallback (coupled=False:
    momentum equations at fixed pressure; coupled=True: full local
    velocity-pressure systems)."""
    bx = _box(box)
    nf = fine_nodes(bx)
    x = _f64(x).reshape(4, nf)
    vprev = _f64(vprev).reshape(3, nf)
    fmid = None if fmid is None else _f64(fmid).reshape(3, nf)
    out = np.zeros((4, nf))
    rc = lib().or_vanka_sweep(ctypes.byref(bx), ctypes.byref(_ns(ns)), _dp(x), _dp(vprev), _dp(fmid),
                              ctypes.c_double(omega), ctypes.c_int(int(coupled)), _dp(out))
    if rc:
        raise np.linalg.LinAlgError("singular local matrix")
    return out
