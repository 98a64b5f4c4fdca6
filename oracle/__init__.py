"""FP64 CPU oracle (ctypes binding to oracle.c).

TEST INFRASTRUCTURE ONLY: the plain, slow definition of the reconstruction
method that the HIP library is checked against.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import this package.  It shares
no code with the HIP library and never imports it.

All arrays are float64, C-contiguous: volumes [nz][ny][nx], DVFs [3][nz][ny][nx],
eigenvector fields [K][3][nz][ny][nx], projections [nv][nu].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, ENOCONV, EDIVERGE = 0, -4, -5


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain double arithmetic, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Grid(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("sp", C.c_double * 3), ("org", C.c_double * 3)]


class _Geom(C.Structure):
    _fields_ = [("angle", C.c_double), ("sad", C.c_double), ("sdd", C.c_double),
                ("nu", C.c_int), ("nv", C.c_int), ("du", C.c_double), ("dv", C.c_double),
                ("off_u", C.c_double), ("off_v", C.c_double), ("step", C.c_double),
                ("iso", C.c_double * 3)]


class _Opts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("max_backtracks", C.c_int), ("sigma", C.c_double),
                ("beta", C.c_double), ("eps_g", C.c_double), ("step0", C.c_double),
                ("fixed_mu", C.c_double), ("mu0", C.c_double), ("step_rule", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("trials", C.c_int), ("status", C.c_int),
                ("J0", C.c_double), ("J", C.c_double), ("gnorm0", C.c_double),
                ("gnorm", C.c_double), ("a", C.c_double), ("b", C.c_double), ("mu", C.c_double)]


_lib = None
_PD = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = C.CDLL(_LIB_PATH)
        G, Gm = C.POINTER(_Grid), C.POINTER(_Geom)
        sig = {
            "orc_num_threads": (C.c_int, []),
            "orc_set_num_threads": (None, [C.c_int]),
            "orc_interp": (C.c_double, [_PD, C.POINTER(C.c_int), _PD]),
            "orc_interp_grad": (None, [_PD, C.POINTER(C.c_int), _PD, _PD]),
            "orc_compose": (None, [G, C.c_int, _PD, _PD, _PD, _PD]),
            "orc_warp": (None, [G, _PD, _PD, _PD]),
            "orc_warp_adjoint": (None, [G, _PD, _PD, _PD]),
            "orc_warp_jacobian": (None, [G, _PD, _PD, _PD]),
            "orc_source_pixel": (None, [Gm, C.c_int, C.c_int, _PD, _PD]),
            "orc_project_ray": (C.c_double, [G, Gm, _PD, C.c_int, C.c_int]),
            "orc_project": (None, [G, Gm, _PD, _PD]),
            "orc_backproject": (None, [G, Gm, _PD, _PD]),
            "orc_regression_sums": (None, [C.c_int, _PD, _PD, _PD]),
            "orc_step2": (None, [_PD, _PD]),
            "orc_cost": (C.c_double, [C.c_int, _PD, _PD, C.c_double, C.c_double, _PD]),
            "orc_cost_grad": (C.c_double, [G, Gm, _PD, C.c_int, _PD, _PD, _PD, _PD,
                                           C.c_double, C.c_double, _PD, _PD]),
            "orc_solve": (C.c_int, [G, Gm, _PD, C.c_int, _PD, _PD, _PD, C.POINTER(_Opts),
                                    _PD, _PD, C.POINTER(_Stats), _PD]),
            "orc_localize": (C.c_int, [G, C.c_int, _PD, _PD, _PD, _PD, C.c_double, C.c_int,
                                       _PD, C.POINTER(C.c_int)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _arr(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def _p(a):
    return a.ctypes.data_as(_PD) if a is not None else None


def _grid(grid) -> _Grid:
    g = _Grid()
    g.n[:] = list(grid.n)
    g.sp[:] = list(grid.spacing)
    g.org[:] = list(grid.origin)
    return g


def _geom(geom) -> _Geom:
    G = _Geom()
    G.angle, G.sad, G.sdd = geom.angle, geom.sad, geom.sdd
    G.nu, G.nv, G.du, G.dv = geom.nu, geom.nv, geom.du, geom.dv
    G.off_u, G.off_v, G.step = geom.off_u, geom.off_v, geom.step
    G.iso[:] = list(geom.iso)
    return G


def _n(grid):
    return (C.c_int * 3)(*grid.n)


# ------------------------------------------------------------ wrappers -----
def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's later parallel regions."""
    _load().orc_set_num_threads(int(n))


def interp(F, grid, q):
    F = _arr(F)
    q = _arr(q)
    return _load().orc_interp(_p(F), _n(grid), _p(q))


def interp_grad(F, grid, q):
    F = _arr(F)
    q = _arr(q)
    out = np.zeros(3)
    _load().orc_interp_grad(_p(F), _n(grid), _p(q), _p(out))
    return out


def compose(grid, mean, U, w):
    K = len(w)
    mean = _arr(mean, (3,) + grid.shape)
    U = _arr(U, (K, 3) + grid.shape)
    w = _arr(w)
    x = np.empty((3,) + grid.shape)
    _load().orc_compose(C.byref(_grid(grid)), K, _p(mean), _p(U), _p(w), _p(x))
    return x


def warp(grid, f0, x):
    f0 = _arr(f0, grid.shape)
    x = _arr(x, (3,) + grid.shape)
    f = np.empty(grid.shape)
    _load().orc_warp(C.byref(_grid(grid)), _p(f0), _p(x), _p(f))
    return f


def warp_adjoint(grid, x, gv):
    x = _arr(x, (3,) + grid.shape)
    gv = _arr(gv, grid.shape)
    out = np.empty(grid.shape)
    _load().orc_warp_adjoint(C.byref(_grid(grid)), _p(x), _p(gv), _p(out))
    return out


def warp_jacobian(grid, f0, x):
    f0 = _arr(f0, grid.shape)
    x = _arr(x, (3,) + grid.shape)
    G = np.empty((3,) + grid.shape)
    _load().orc_warp_jacobian(C.byref(_grid(grid)), _p(f0), _p(x), _p(G))
    return G


def source_pixel(geom, iu, iv):
    s, pix = np.zeros(3), np.zeros(3)
    _load().orc_source_pixel(C.byref(_geom(geom)), iu, iv, _p(s), _p(pix))
    return s, pix


def project_ray(grid, geom, f, iu, iv):
    f = _arr(f, grid.shape)
    return _load().orc_project_ray(C.byref(_grid(grid)), C.byref(_geom(geom)), _p(f), iu, iv)


def project(grid, geom, f):
    f = _arr(f, grid.shape)
    p = np.empty((geom.nv, geom.nu))
    _load().orc_project(C.byref(_grid(grid)), C.byref(_geom(geom)), _p(f), _p(p))
    return p


def backproject(grid, geom, r):
    r = _arr(r, (geom.nv, geom.nu))
    out = np.empty(grid.shape)
    _load().orc_backproject(C.byref(_grid(grid)), C.byref(_geom(geom)), _p(r), _p(out))
    return out


def regression_sums(y, p):
    y, p = _arr(y).ravel(), _arr(p).ravel()
    S = np.zeros(5)
    _load().orc_regression_sums(y.size, _p(y), _p(p), _p(S))
    return S


def step2(S):
    S = _arr(S)
    ab = np.zeros(2)
    _load().orc_step2(_p(S), _p(ab))
    return float(ab[0]), float(ab[1])


def cost(p, y, a, b, want_r=False):
    p, y = _arr(p), _arr(y)
    r = np.empty_like(p) if want_r else None
    J = _load().orc_cost(p.size, _p(p), _p(y), a, b, _p(r))
    return (J, r) if want_r else J


def cost_grad(grid, geom, f0, mean, U, w, y, a, b, want_p=False):
    K = len(w)
    f0 = _arr(f0, grid.shape)
    mean = _arr(mean, (3,) + grid.shape)
    U = _arr(U, (K, 3) + grid.shape)
    w, y = _arr(w), _arr(y, (geom.nv, geom.nu))
    grad = np.zeros(K)
    p = np.empty((geom.nv, geom.nu)) if want_p else None
    J = _load().orc_cost_grad(C.byref(_grid(grid)), C.byref(_geom(geom)), _p(f0), K, _p(mean),
                              _p(U), _p(w), _p(y), a, b, _p(grad), _p(p))
    return (J, grad, p) if want_p else (J, grad)


@dataclass
class SolveOpts:
    max_iter: int = 30
    max_backtracks: int = 30
    sigma: float = 1e-4
    beta: float = 0.5
    eps_g: float = 1e-4
    step0: float = 1.0
    fixed_mu: float = 0.0
    mu0: float = 0.0
    step_rule: int = 0        # later first trials: 0 secant, 1 quadratic model


def solve(grid, geom, f0, mean, U, y, w0, opts: SolveOpts):
    """Runs the alternating algorithm; returns (w, (a, b), stats dict, J history)."""
    K = len(w0)
    f0 = _arr(f0, grid.shape)
    mean = _arr(mean, (3,) + grid.shape)
    U = _arr(U, (K, 3) + grid.shape)
    y = _arr(y, (geom.nv, geom.nu))
    w = np.array(w0, dtype=np.float64, copy=True)
    ab = np.zeros(2)
    o = _Opts(opts.max_iter, opts.max_backtracks, opts.sigma, opts.beta, opts.eps_g,
              opts.step0, opts.fixed_mu, opts.mu0, opts.step_rule)
    st = _Stats()
    Jh = np.full(opts.max_iter + 1, np.nan)
    _load().orc_solve(C.byref(_grid(grid)), C.byref(_geom(geom)), _p(f0), K, _p(mean), _p(U),
                      _p(y), C.byref(o), _p(w), _p(ab), C.byref(st), _p(Jh))
    stats = {k: getattr(st, k) for k, _ in _Stats._fields_}
    return w, (float(ab[0]), float(ab[1])), stats, Jh[: st.iterations + 1]


def localize(grid, mean, U, w, p_ref, tol=1e-6, max_iter=200):
    K = len(w)
    mean = _arr(mean, (3,) + grid.shape)
    U = _arr(U, (K, 3) + grid.shape)
    w, p_ref = _arr(w), _arr(p_ref)
    out = np.zeros(3)
    it = C.c_int(0)
    st = _load().orc_localize(C.byref(_grid(grid)), K, _p(mean), _p(U), _p(w), _p(p_ref),
                              tol, max_iter, _p(out), C.byref(it))
    return out, st, it.value


def pca(dvfs, K):
    """PCA of the motion model (section 2.1, eq. (1); section 3): dvfs
    [J][3][...] training DVFs.  mean = their average; U = the K leading left
    singular vectors of the centred 3N x J matrix (numpy SVD, float64), each
    flipped so that its first entry within 1e-5 (relative) of its largest
    magnitude is positive; w_train[j][k] = <U_k, d_j - mean>.  Returns
    (mean, U, singular values, w_train)."""
    d = np.asarray(dvfs, dtype=np.float64)
    J = d.shape[0]
    X = d.reshape(J, -1).T                       # 3N x J
    mean = X.mean(axis=1)
    Xc = X - mean[:, None]
    u, s, _ = np.linalg.svd(Xc, full_matrices=False)
    U = u[:, :K].copy()
    for k in range(K):
        a = np.abs(U[:, k])
        j = int(np.flatnonzero(a >= (1 - 1e-5) * a.max())[0])
        if U[j, k] < 0:
            U[:, k] = -U[:, k]
    w_train = Xc.T @ U
    shape = d.shape[1:]
    return mean.reshape(shape), U.T.reshape((K,) + shape), s[:K], w_train
