"""ctypes binding of libpcr.so (include/pcr.h): argument marshalling only.

Every computation runs in the HIP library; torch supplies device memory and
the current stream.  Importing this module does not load the library; the
first call does, and raises if it has not been built (there is no CPU path).
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcr.so")

PCR_OK, PCR_EINVAL, PCR_ENOMEM, PCR_EDEVICE, PCR_ENOCONV, PCR_EDIVERGE, PCR_EBUSY = 0, -1, -2, -3, -4, -5, -6
PCR_F32, PCR_F64, PCR_BF16, PCR_F16 = 0, 1, 2, 3
PCR_STEP_SECANT, PCR_STEP_QUADRATIC = 0, 1
GRAD_FUSED, GRAD_ADJOINT = 0, 1

_DT = {torch.float32: PCR_F32, torch.float64: PCR_F64, torch.bfloat16: PCR_BF16,
       torch.float16: PCR_F16}


class PCRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("pcr status %d: %s" % (status, msg))
        self.status = status


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("spacing_mm", C.c_double * 3), ("origin_mm", C.c_double * 3)]


class Geom(C.Structure):
    _fields_ = [("angle_rad", C.c_double), ("sad_mm", C.c_double), ("sdd_mm", C.c_double),
                ("nu", C.c_int32), ("nv", C.c_int32), ("du_mm", C.c_double), ("dv_mm", C.c_double),
                ("off_u_mm", C.c_double), ("off_v_mm", C.c_double), ("step_mm", C.c_double),
                ("iso_mm", C.c_double * 3)]


class Model(C.Structure):
    _fields_ = [("K", C.c_int32), ("storage", C.c_int), ("mean", C.c_void_p), ("U", C.c_void_p),
                ("scale", C.POINTER(C.c_double))]


class SolveOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("max_backtracks", C.c_int32), ("sigma", C.c_double),
                ("beta", C.c_double), ("eps_g", C.c_double), ("step0", C.c_double),
                ("fixed_mu", C.c_double), ("grad_mode", C.c_int32), ("localize", C.c_int32),
                ("p_ref_mm", C.c_double * 3), ("fp_tol_mm", C.c_double), ("fp_max_iter", C.c_int32),
                ("mu0", C.c_double), ("step_rule", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("trials", C.c_int32),
                ("fp_iterations", C.c_int32), ("fp_status", C.c_int32), ("J0", C.c_double),
                ("J", C.c_double), ("gnorm0", C.c_double), ("gnorm", C.c_double),
                ("a", C.c_double), ("b", C.c_double), ("tumor_mm", C.c_double * 3),
                ("samples", C.c_double), ("mu", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["tumor_mm"] = list(self.tumor_mm)
        return d


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32), ("drop_stale", C.c_int32),
                ("predict_order", C.c_int32), ("chain_step", C.c_int32), ("image_f16", C.c_int32),
                ("carry_move", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("req_id", C.c_int64), ("stream_id", C.c_int32), ("status", C.c_int32),
                ("iterations", C.c_int32), ("trials", C.c_int32), ("K", C.c_int32),
                ("fp_status", C.c_int32), ("w0", C.c_double * 8), ("w", C.c_double * 8),
                ("ab", C.c_double * 2), ("J", C.c_double), ("tumor_mm", C.c_double * 3),
                ("t_submit_s", C.c_double), ("t_start_s", C.c_double), ("t_done_s", C.c_double),
                ("mu0", C.c_double), ("mu", C.c_double), ("samples", C.c_double),
                ("step0", C.c_double)]

    def as_dict(self):
        K = self.K
        return {"req_id": self.req_id, "stream_id": self.stream_id, "status": self.status,
                "iterations": self.iterations, "trials": self.trials, "fp_status": self.fp_status,
                "w0": list(self.w0[:K]), "w": list(self.w[:K]), "ab": list(self.ab), "J": self.J,
                "tumor_mm": list(self.tumor_mm), "t_submit_s": self.t_submit_s,
                "t_start_s": self.t_start_s, "t_done_s": self.t_done_s, "mu0": self.mu0,
                "mu": self.mu, "samples": self.samples, "step0": self.step0}


_lib = None
_P = C.c_void_p
_PD = C.POINTER(C.c_double)


def lib():
    """The loaded library; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built; run "
                               "`python -m paper_1004_0014_amd.build`" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        G, Gm, Md = C.POINTER(Grid), C.POINTER(Geom), C.POINTER(Model)
        sig = {
            "pcr_version": (C.c_char_p, []),
            "pcr_last_error": (C.c_char_p, []),
            "pcr_solve_opts_default": (None, [C.POINTER(SolveOpts)]),
            "pcr_dvf_compose": (C.c_int32, [G, Md, _PD, C.c_int, _P, _P]),
            "pcr_warp_volume": (C.c_int32, [G, C.c_int, _P, C.c_int, _P, _P, _P]),
            "pcr_warp_adjoint": (C.c_int32, [G, C.c_int, _P, _P, _P, _P]),
            "pcr_forward_project": (C.c_int32, [G, Gm, C.c_int, _P, _P, _P]),
            "pcr_forward_project_noalloc": (C.c_int32, [G, Gm, C.c_int, _P, _P, _P]),
            "pcr_backproject_residual": (C.c_int32, [G, Gm, C.c_int, _P, _P, _P]),
            "pcr_ctx_create": (C.c_int32, [G, Md, C.c_int, _P, C.c_int, C.POINTER(_P)]),
            "pcr_ctx_destroy": (None, [_P]),
            "pcr_ctx_device_bytes": (C.c_size_t, [_P]),
            "pcr_ctx_set_image_dtype": (C.c_int32, [_P, C.c_int]),
            "pcr_cost_grad": (C.c_int32, [_P, _P, Gm, _PD, C.c_double, C.c_double, C.c_int32,
                                          _PD, _PD, _P]),
            "pcr_reconstruct_from_projection": (C.c_int32, [_P, _P, Gm, C.POINTER(SolveOpts), _PD,
                                                            _PD, C.POINTER(SolveStats), _P]),
            "pcr_localize_tumor": (C.c_int32, [G, Md, _PD, _PD, C.c_double, C.c_int32, _PD,
                                               C.POINTER(C.c_int32), _P]),
            "pcr_warp_contract": (C.c_int32, [G, Md, C.c_int, _P, _PD, C.c_int, _P, _PD, _P]),
            "pcr_server_create": (C.c_int32, [C.POINTER(ServerOpts), C.POINTER(_P)]),
            "pcr_server_destroy": (None, [_P]),
            "pcr_server_add_stream": (C.c_int32, [_P, G, Md, C.c_int, _P, C.POINTER(SolveOpts), _PD,
                                                  C.POINTER(C.c_int32)]),
            "pcr_server_remove_stream": (C.c_int32, [_P, C.c_int32]),
            "pcr_server_submit": (C.c_int32, [_P, C.c_int32, _P, Gm, C.POINTER(C.c_int64)]),
            "pcr_server_poll": (C.c_int32, [_P, C.POINTER(Result), C.c_int32, C.POINTER(C.c_int32),
                                            C.c_int32]),
            "pcr_server_drain": (C.c_int32, [_P, C.c_int32]),
            "pcr_server_get_w": (C.c_int32, [_P, C.c_int32, _PD]),
            "pcr_server_set_w": (C.c_int32, [_P, C.c_int32, _PD]),
            "pcr_server_device_bytes": (C.c_size_t, [_P]),
            "pcr_predict_w": (C.c_int32, [_PD, _PD, C.c_int32, C.c_int32, C.c_double, C.c_int32, _PD]),
            "pcr_pca_train": (C.c_int32, [G, C.c_int32, _P, C.c_int32, _P, _P, _PD, _PD, _P]),
            "pcr_profile_enable": (None, [C.c_int32]),
            "pcr_profile_select": (None, [C.c_uint32]),
            "pcr_profile_read": (C.c_int32, [C.c_int32, C.POINTER(C.c_char_p), _PD,
                                             C.POINTER(C.c_int64)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def version() -> str:
    return lib().pcr_version().decode()


def _check(st, ok=(PCR_OK,)):
    if st not in ok:
        raise PCRError(st, lib().pcr_last_error().decode())
    return st


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _dtype(t: torch.Tensor) -> int:
    try:
        return _DT[t.dtype]
    except KeyError:
        raise ValueError("unsupported dtype %s" % t.dtype)


def _dd(seq):
    arr = (C.c_double * len(seq))(*[float(v) for v in seq])
    return arr


def make_grid(grid) -> Grid:
    """From any object with n (nx, ny, nz), spacing and origin (mm)."""
    g = Grid()
    g.n[:] = [int(v) for v in grid.n]
    g.spacing_mm[:] = [float(v) for v in grid.spacing]
    g.origin_mm[:] = [float(v) for v in grid.origin]
    return g


def make_geom(geom) -> Geom:
    """From any object with angle, sad, sdd, nu, nv, du, dv, off_u, off_v,
    step and iso."""
    G = Geom()
    G.angle_rad, G.sad_mm, G.sdd_mm = geom.angle, geom.sad, geom.sdd
    G.nu, G.nv, G.du_mm, G.dv_mm = geom.nu, geom.nv, geom.du, geom.dv
    G.off_u_mm, G.off_v_mm, G.step_mm = geom.off_u, geom.off_v, geom.step
    G.iso_mm[:] = [float(v) for v in geom.iso]
    return G


class DeviceModel:
    """Device-resident motion model: mean [3][N] and U [K][3][N] of one
    storage dtype, and optional per-field scales (field k = scale_k U_k)."""

    def __init__(self, mean: torch.Tensor, U: torch.Tensor, scale=None):
        if mean.dtype != U.dtype:
            raise ValueError("mean and U must share a dtype")
        self.mean = mean.contiguous()
        self.U = U.contiguous()
        self.K = int(U.shape[0])
        self.scale = None if scale is None else [float(s) for s in scale]
        self._scale_arr = None if scale is None else _dd(self.scale)
        self.struct = Model(self.K, _dtype(self.mean), _ptr(self.mean).value, _ptr(self.U).value,
                            C.cast(self._scale_arr, _PD) if scale is not None else None)


# --------------------------------------------------------------- calls -----
def dvf_compose(grid, model: DeviceModel, w, compute=torch.float32, stream=None):
    g = make_grid(grid)
    nx, ny, nz = g.n
    out = torch.empty((3, nz, ny, nx), dtype=compute, device=model.mean.device)
    _check(lib().pcr_dvf_compose(C.byref(g), C.byref(model.struct), _dd(w), _DT[compute],
                                 _ptr(out), _stream(stream)))
    return out


def warp_volume(grid, f0: torch.Tensor, dvf: torch.Tensor, stream=None):
    g = make_grid(grid)
    out = torch.empty(f0.shape, dtype=dvf.dtype, device=f0.device)
    _check(lib().pcr_warp_volume(C.byref(g), _dtype(f0), _ptr(f0), _dtype(dvf), _ptr(dvf), _ptr(out),
                                 _stream(stream)))
    return out


def warp_adjoint(grid, dvf: torch.Tensor, gvol: torch.Tensor, stream=None):
    g = make_grid(grid)
    out = torch.empty(gvol.shape, dtype=gvol.dtype, device=gvol.device)
    _check(lib().pcr_warp_adjoint(C.byref(g), _dtype(dvf), _ptr(dvf), _ptr(gvol), _ptr(out),
                                  _stream(stream)))
    return out


def forward_project(grid, geom, vol: torch.Tensor, out=None, stream=None):
    g, G = make_grid(grid), make_geom(geom)
    if out is None:
        out = torch.empty((G.nv, G.nu), dtype=vol.dtype, device=vol.device)
    _check(lib().pcr_forward_project(C.byref(g), C.byref(G), _dtype(vol), _ptr(vol), _ptr(out),
                                     _stream(stream)))
    return out


def forward_project_noalloc(grid, geom, vol: torch.Tensor, out: torch.Tensor, stream=None):
    """pcr_forward_project_noalloc: the caller passes the output too."""
    g, G = make_grid(grid), make_geom(geom)
    if tuple(out.shape) != (G.nv, G.nu) or out.dtype != vol.dtype:
        raise ValueError("out must be [nv][nu] of the volume's dtype")
    if vol.numel() != g.n[0] * g.n[1] * g.n[2]:
        raise ValueError("vol must hold nx*ny*nz values")
    _check(lib().pcr_forward_project_noalloc(C.byref(g), C.byref(G), _dtype(vol), _ptr(vol),
                                             _ptr(out), _stream(stream)))
    return out


def backproject_residual(grid, geom, resid: torch.Tensor, out=None, stream=None):
    g, G = make_grid(grid), make_geom(geom)
    nx, ny, nz = g.n
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=resid.dtype, device=resid.device)
    _check(lib().pcr_backproject_residual(C.byref(g), C.byref(G), _dtype(resid), _ptr(resid),
                                          _ptr(out), _stream(stream)))
    return out


def warp_contract(grid, model: DeviceModel, f0: torch.Tensor, w, gvol: torch.Tensor, stream=None):
    """[K] list: scale_k sum_v g[v] (df/dx)[v] . U_k[v] at the DVF for w."""
    g = make_grid(grid)
    out = (C.c_double * model.K)()
    _check(lib().pcr_warp_contract(C.byref(g), C.byref(model.struct), _dtype(f0), _ptr(f0), _dd(w),
                                   _dtype(gvol), _ptr(gvol), out, _stream(stream)))
    return [out[k] for k in range(model.K)]


def pca_train(grid, dvfs: torch.Tensor, K: int, stream=None):
    """GPU PCA of J training DVFs [J][3][nz][ny][nx] (FP32): returns (mean,
    U, singular values, w_train [J][K])."""
    import numpy as np
    g = make_grid(grid)
    J = int(dvfs.shape[0])
    mean = torch.empty(dvfs.shape[1:], dtype=torch.float32, device=dvfs.device)
    U = torch.empty((K,) + tuple(dvfs.shape[1:]), dtype=torch.float32, device=dvfs.device)
    sing = (C.c_double * K)()
    wt = (C.c_double * (J * K))()
    _check(lib().pcr_pca_train(C.byref(g), J, _ptr(dvfs), K, _ptr(mean), _ptr(U), sing, wt,
                               _stream(stream)))
    return mean, U, np.array(list(sing)), np.array(list(wt)).reshape(J, K)


def predict_w(w_hist, t_hist, t_next, order=1):
    """Initial guess extrapolated from previous results (host only)."""
    import numpy as np
    wh = np.ascontiguousarray(w_hist, dtype=np.float64)
    n, K = wh.shape
    out = (C.c_double * K)()
    _check(lib().pcr_predict_w(_dd(wh.ravel()), _dd(t_hist), n, K, float(t_next), int(order), out))
    return list(out)


def localize_tumor(grid, model: DeviceModel, w, p_ref, tol=1e-6, max_iter=200, stream=None):
    """Returns (position mm [3], status, iterations)."""
    g = make_grid(grid)
    out = (C.c_double * 3)()
    it = C.c_int32(0)
    st = lib().pcr_localize_tumor(C.byref(g), C.byref(model.struct), _dd(w), _dd(p_ref), tol,
                                  max_iter, out, C.byref(it), _stream(stream))
    _check(st, ok=(PCR_OK, PCR_EDIVERGE))
    return [out[0], out[1], out[2]], st, it.value


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().pcr_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "p_ref_mm":
            o.p_ref_mm[:] = [float(x) for x in v]
        else:
            setattr(o, k, v)
    return o


class Context:
    """Solver context (pcr_ctx): binds grid, model and reference image."""

    def __init__(self, grid, model: DeviceModel, f0: torch.Tensor, compute=torch.float32,
                 image_dtype=torch.float32):
        self.grid = grid
        self.model = model
        self.f0 = f0.contiguous()
        self.compute = compute
        self.K = model.K
        self._g = make_grid(grid)
        h = C.c_void_p()
        _check(lib().pcr_ctx_create(C.byref(self._g), C.byref(model.struct), _dtype(self.f0),
                                    _ptr(self.f0), _DT[compute], C.byref(h)))
        self._h = h
        if image_dtype != torch.float32:
            _check(lib().pcr_ctx_set_image_dtype(self._h, _DT[image_dtype]))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pcr_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def device_bytes(self) -> int:
        return lib().pcr_ctx_device_bytes(self._h)

    def cost_grad(self, y: torch.Tensor, geom, w, a, b, mode=GRAD_FUSED, stream=None):
        G = make_geom(geom)
        J = C.c_double(0)
        grad = (C.c_double * self.K)()
        _check(lib().pcr_cost_grad(self._h, _ptr(y), C.byref(G), _dd(w), float(a), float(b), mode,
                                   C.byref(J), grad, _stream(stream)))
        return J.value, [grad[k] for k in range(self.K)]

    def reconstruct(self, y: torch.Tensor, geom, w0, opts: SolveOpts, stream=None):
        """Returns (w, (a, b), stats dict)."""
        G = make_geom(geom)
        w = _dd(w0)
        ab = (C.c_double * 2)()
        st = SolveStats()
        _check(lib().pcr_reconstruct_from_projection(self._h, _ptr(y), C.byref(G), C.byref(opts), w, ab,
                                                     C.byref(st), _stream(stream)),
               ok=(PCR_OK, PCR_ENOCONV))
        return [w[k] for k in range(self.K)], (ab[0], ab[1]), st.as_dict()


PROFILE_KINDS = ("warp_fused", "march", "reduce", "backproject", "contract", "localize", "zero", "pad",
                 "unpad", "compose", "warp", "warp_adjoint", "pca_gram", "pca_fields")


def profile_enable(on: bool = True, kinds=None):
    """Per-kernel HIP-event timing inside the library (resets when enabled),
    of every kernel kind or only of `kinds` (names as profile_read reports)."""
    mask = 0xFFFFFFFF if kinds is None else sum(1 << PROFILE_KINDS.index(k) for k in kinds)
    lib().pcr_profile_select(mask)
    lib().pcr_profile_enable(1 if on else 0)


def profile_read() -> dict:
    """{kernel: (total_ms, launches)} for kernels launched while enabled."""
    n = 32
    names = (C.c_char_p * n)()
    tot = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    k = lib().pcr_profile_read(n, names, tot, cnt)
    return {names[i].decode(): (tot[i], cnt[i]) for i in range(min(k, n)) if cnt[i] > 0}


class Server:
    """Serving engine (pcr_server_*): continuous batching of per-projection
    solves for many streams.  Streams' reference images and models are copied
    into server-owned device memory at add_stream."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 8, drop_stale: bool = True,
                 predict_order: int = 0, chain_step: bool = False, image_f16: bool = False,
                 carry_move: bool = False):
        o = ServerOpts(int(hbm_budget_bytes), int(max_slots), 1 if drop_stale else 0, int(predict_order),
                       1 if chain_step else 0, 1 if image_f16 else 0, 1 if carry_move else 0)
        h = C.c_void_p()
        _check(lib().pcr_server_create(C.byref(o), C.byref(h)))
        self._h = h
        self._geoms = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pcr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_stream(self, grid, model: DeviceModel, f0: torch.Tensor, opts: SolveOpts, w0) -> int:
        """Returns the stream id; raises PCRError with status PCR_EBUSY when
        the HBM budget would be exceeded."""
        g = make_grid(grid)
        sid = C.c_int32(-1)
        _check(lib().pcr_server_add_stream(self._h, C.byref(g), C.byref(model.struct), _dtype(f0),
                                           _ptr(f0), C.byref(opts), _dd(w0), C.byref(sid)))
        return sid.value

    def remove_stream(self, sid: int):
        _check(lib().pcr_server_remove_stream(self._h, sid))

    def submit(self, sid: int, y: torch.Tensor, geom) -> int:
        G = make_geom(geom)
        rid = C.c_int64(-1)
        _check(lib().pcr_server_submit(self._h, sid, _ptr(y), C.byref(G), C.byref(rid)))
        return rid.value

    def poll(self, max_results: int = 256, wait_ms: int = 0):
        buf = (Result * max_results)()
        n = C.c_int32(0)
        _check(lib().pcr_server_poll(self._h, buf, max_results, C.byref(n), wait_ms))
        return [buf[i].as_dict() for i in range(n.value)]

    def drain(self, timeout_ms: int = -1):
        _check(lib().pcr_server_drain(self._h, timeout_ms))

    def get_w(self, sid: int, K: int):
        w = (C.c_double * K)()
        _check(lib().pcr_server_get_w(self._h, sid, w))
        return list(w)

    def set_w(self, sid: int, w):
        _check(lib().pcr_server_set_w(self._h, sid, _dd(w)))

    @property
    def device_bytes(self) -> int:
        return lib().pcr_server_device_bytes(self._h)
