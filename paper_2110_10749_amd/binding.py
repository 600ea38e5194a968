"""ctypes binding of libsdbie.so: argument marshalling only.

Every computation happens in the HIP library.  torch supplies device memory
(float64 CUDA/HIP tensors) and the current stream.  The names mirror the C
ABI in include/sdbie.h.  The library must have been built
(`python -m paper_2110_10749_amd.build`); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdbie.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_NONFINITE, ERR_DEVICE, ERR_WORKSPACE = -1, -2, -3, -4
FP64, MIXED = 0, 1
SL, DL_RAW, DL_SUB = 0, 1, 2

_PREC = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}
_LAYER = {"sl": SL, "dl_raw": DL_RAW, "dl_sub": DL_SUB, SL: SL, DL_RAW: DL_RAW, DL_SUB: DL_SUB}


class SdbieError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sdbie error {code}: {msg}")
        self.code = code


class Surface(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("nrm", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("delta", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("K", ctypes.c_double), ("alpha", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("tol_gmres", ctypes.c_double), ("tol_ddm", ctypes.c_double), ("theta", ctypes.c_double),
                ("maxit_gmres", ctypes.c_int), ("restart", ctypes.c_int), ("maxit_ddm", ctypes.c_int),
                ("outer", ctypes.c_int), ("slip", ctypes.c_int), ("prec", ctypes.c_int),
                ("tol_mixed", ctypes.c_double), ("refine_max", ctypes.c_int), ("mixed_mode", ctypes.c_int),
                ("relax_outer", ctypes.c_int), ("local_solver", ctypes.c_int), ("recycle", ctypes.c_int)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("pairs", ctypes.c_double), ("flops_per_pair", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("ddm_iters", ctypes.c_int), ("gmres_iters", ctypes.c_int), ("refine_steps", ctypes.c_int),
                ("applies_fp64", ctypes.c_int64), ("applies_mixed", ctypes.c_int64), ("pairs", ctypes.c_double),
                ("ddm_res", ctypes.c_double), ("relres", ctypes.c_double)]

    def as_dict(self, status: int = OK) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["converged"] = status == OK
        return d


_lib = None
ABI_VERSION = 4  # layout of the structs above (sdbie_abi_version)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2110_10749_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.sdbie_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.sdbie_default_opts.restype = None
        L.sdbie_workspace_bytes.argtypes = [i64, i32]
        L.sdbie_workspace_bytes.restype = ctypes.c_size_t
        L.sdbie_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Surface), i32, vp, ctypes.c_size_t, vp]
        L.sdbie_plan_create.restype = i32
        L.sdbie_plan_destroy.argtypes = [vp]
        L.sdbie_plan_destroy.restype = i32
        L.sdbie_plan_n.argtypes = [vp]
        L.sdbie_plan_n.restype = i64
        L.sdbie_plan_set_symmetric.argtypes = [vp, i32]
        L.sdbie_plan_set_symmetric.restype = i32
        L.laplace_layer_apply.argtypes = [vp, i32, vp, vp, i32, vp]
        L.laplace_layer_apply.restype = i32
        L.stokes_layer_apply.argtypes = [vp, d, i32, vp, vp, i32, vp]
        L.stokes_layer_apply.restype = i32
        L.stokes_layer_apply_noalloc.argtypes = [ctypes.POINTER(Surface), d, i32, vp, vp, i32, vp]
        L.stokes_layer_apply_noalloc.restype = i32
        L.darcy_solve.argtypes = [vp, ctypes.POINTER(Params), vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(Info), vp]
        L.darcy_solve.restype = i32
        L.stokes_solve.argtypes = [vp, ctypes.POINTER(Params), ctypes.POINTER(d), vp, vp, vp,
                                   ctypes.POINTER(Opts), ctypes.POINTER(Info), vp]
        L.stokes_solve.restype = i32
        L.ddm_solve.argtypes = [vp, ctypes.POINTER(Params), ctypes.POINTER(d), vp, vp, vp, ctypes.POINTER(d),
                                ctypes.POINTER(Opts), ctypes.POINTER(Info), vp]
        L.ddm_solve.restype = i32
        L.ddm_adjoint.argtypes = [vp, ctypes.POINTER(Params), ctypes.POINTER(d), vp, vp, vp, ctypes.POINTER(d), vp,
                                  ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(Opts), ctypes.POINTER(Info), vp]
        L.ddm_adjoint.restype = i32
        L.ddm_dn_spectrum.argtypes = [vp, ctypes.POINTER(Params), vp, i32, i32, ctypes.POINTER(d),
                                      ctypes.POINTER(d), ctypes.POINTER(Opts), ctypes.POINTER(Info), vp]
        L.ddm_dn_spectrum.restype = i32
        L.sdbie_hessenberg_eigenvalues.argtypes = [i32, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d)]
        L.sdbie_hessenberg_eigenvalues.restype = i32
        L.sdbie_last_error.argtypes = []
        L.sdbie_last_error.restype = ctypes.c_char_p
        L.sdbie_abi_version.argtypes = []
        L.sdbie_abi_version.restype = i32
        L.sdbie_profile_enable.argtypes = [i32]
        L.sdbie_profile_enable.restype = i32
        L.sdbie_profile_read.argtypes = [ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
        L.sdbie_profile_read.restype = i32
        if L.sdbie_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI {L.sdbie_abi_version()}, this binding needs {ABI_VERSION}: "
                              f"rebuild it")
        _lib = L
    return _lib


def _check(code: int, allow_not_converged: bool = True) -> int:
    if code < 0 or (code == NOT_CONVERGED and not allow_not_converged):
        raise SdbieError(code, lib().sdbie_last_error().decode())
    return code


def _dev(t: torch.Tensor, shape, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def profile_enable(on: bool = True) -> None:
    """Start (and clear) or stop the per-kernel HIP-event timing of pair-sum launches."""
    _check(lib().sdbie_profile_enable(1 if on else 0))


def profile_read() -> list:
    """Per-variant kernel timing recorded since profile_enable(True) (waits for the events)."""
    cnt = ctypes.c_int(0)
    _check(lib().sdbie_profile_read(None, 0, ctypes.byref(cnt)))
    arr = (KernelStat * max(cnt.value, 1))()
    _check(lib().sdbie_profile_read(arr, cnt.value, ctypes.byref(cnt)))
    return [dict(name=a.name.decode(), launches=a.launches, ms=a.ms, pairs=a.pairs,
                 flops_per_pair=a.flops_per_pair) for a in arr[:cnt.value]]


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().sdbie_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "prec":
            v = _PREC[v]
        if k == "outer" and isinstance(v, str):
            v = {"sa": 0, "gmres": 1}[v]
        if k == "slip" and isinstance(v, str):
            v = {"implicit": 0, "lagged": 1}[v]
        if k == "mixed_mode" and isinstance(v, str):
            v = {"refine": 0, "coupled": 1, "relaxed": 2}[v]
        if k == "local_solver" and isinstance(v, str):
            v = {"gmres": 0, "sa": 1}[v]
        setattr(o, k, v)
    return o


def workspace_bytes(n: int, max_restart: int = 50) -> int:
    return int(lib().sdbie_workspace_bytes(n, max_restart))


# pass kinds of sdbie_plan_set_symmetric (SDBIE_SYM_*): float-pair and double-pair passes
SYM_LAPLACE = 1
SYM_STOKES = 2
SYM_LAPLACE_F64 = 4
SYM_STOKES_F64 = 8
SYM_ALL = 15
SYM_DEFAULT = SYM_LAPLACE | SYM_STOKES | SYM_LAPLACE_F64 | SYM_STOKES_F64


class Plan:
    """A staged surface: node data copied into a device workspace in Morton order.

    x, nrm: float64 device tensors (3, N); w: (N,); delta > 0.
    """

    def __init__(self, x, nrm, w, delta: float, max_restart: int = 50):
        n = int(w.shape[0])
        x = _dev(x, (3, n), "x")
        nrm = _dev(nrm, (3, n), "nrm")
        w = _dev(w, (n,), "w")
        self.device = x.device
        self.n = n
        self.delta = float(delta)
        self.max_restart = int(max_restart)
        nbytes = workspace_bytes(n, max_restart)
        if nbytes == 0:
            raise SdbieError(ERR_ARG, "invalid n or max_restart")
        # over-allocate by 256 bytes and align
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        surf = Surface(n, x.data_ptr(), nrm.data_ptr(), w.data_ptr(), self.delta)
        h = ctypes.c_void_p()
        _check(lib().sdbie_plan_create(ctypes.byref(h), ctypes.byref(surf), self.max_restart,
                                       ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(nbytes),
                                       _stream(self.device)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def set_symmetric(self, kinds=SYM_ALL) -> None:
        """Evaluate the far tile pairs of the selected pass kinds once for both
        directions (sdbie_plan_set_symmetric).  ``kinds``: a mask of
        SYM_LAPLACE, SYM_STOKES (float pairs), SYM_LAPLACE_F64, SYM_STOKES_F64
        (double pairs); True means all, False none.  A new plan starts at
        SYM_DEFAULT."""
        if kinds is True:
            kinds = SYM_ALL
        elif kinds is False:
            kinds = 0
        _check(lib().sdbie_plan_set_symmetric(self._h, int(kinds)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sdbie_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def laplace_layer_apply(plan: Plan, layer, dens, out=None, prec="fp64"):
    dens = _dev(dens, (plan.n,), "dens")
    out = torch.empty_like(dens) if out is None else _dev(out, (plan.n,), "out")
    _check(lib().laplace_layer_apply(plan.handle, _LAYER[layer], _ptr(dens), _ptr(out), _PREC[prec],
                                     _stream(plan.device)))
    return out


def stokes_layer_apply(plan: Plan, mu: float, layer, dens, out=None, prec="fp64"):
    dens = _dev(dens, (3, plan.n), "dens")
    out = torch.empty_like(dens) if out is None else _dev(out, (3, plan.n), "out")
    _check(lib().stokes_layer_apply(plan.handle, float(mu), _LAYER[layer], _ptr(dens), _ptr(out), _PREC[prec],
                                    _stream(plan.device)))
    return out


NOALLOC_MAX_NODES = 32768  # SDBIE_NOALLOC_MAX_NODES


def stokes_layer_apply_noalloc(x, nrm, w, delta: float, mu: float, layer, dens, out=None, prec="fp64"):
    """Stokes layer sum of a surface given directly (no plan, no device allocation in the
    library: the surface is staged into its static device array on every call)."""
    n = int(w.shape[0])
    x = _dev(x, (3, n), "x")
    nrm = _dev(nrm, (3, n), "nrm")
    w = _dev(w, (n,), "w")
    dens = _dev(dens, (3, n), "dens")
    out = torch.empty_like(dens) if out is None else _dev(out, (3, n), "out")
    surf = Surface(n, x.data_ptr(), nrm.data_ptr(), w.data_ptr(), float(delta))
    _check(lib().stokes_layer_apply_noalloc(ctypes.byref(surf), float(mu), _LAYER[layer], _ptr(dens), _ptr(out),
                                            _PREC[prec], _stream(x.device)))
    return out


def _params(mu, K, alpha) -> Params:
    return Params(float(mu), float(K), float(alpha))


def _opts(opts) -> Opts:
    if opts is None:
        return default_opts()
    if isinstance(opts, dict):
        return default_opts(**opts)
    return opts


def darcy_solve(plan: Plan, mu, K, alpha, vn, p=None, opts=None):
    """Returns (p, info dict)."""
    vn = _dev(vn, (plan.n,), "vn")
    p = torch.zeros_like(vn) if p is None else _dev(p, (plan.n,), "p").clone()
    prm, o, info = _params(mu, K, alpha), _opts(opts), Info()
    st = _check(lib().darcy_solve(plan.handle, ctypes.byref(prm), _ptr(vn), _ptr(p), ctypes.byref(o),
                                  ctypes.byref(info), _stream(plan.device)))
    return p, info.as_dict(st)


def stokes_solve(plan: Plan, mu, K, alpha, U, p, f_extra=None, u=None, opts=None):
    """Returns (u, info dict).  U: 3 floats (host)."""
    p = _dev(p, (plan.n,), "p")
    if f_extra is not None:
        f_extra = _dev(f_extra, (3, plan.n), "f_extra")
    u = torch.zeros((3, plan.n), dtype=torch.float64, device=plan.device) if u is None else \
        _dev(u, (3, plan.n), "u").clone()
    Uc = (ctypes.c_double * 3)(*[float(v) for v in U])
    prm, o, info = _params(mu, K, alpha), _opts(opts), Info()
    st = _check(lib().stokes_solve(plan.handle, ctypes.byref(prm), Uc, _ptr(p), _ptr(f_extra), _ptr(u),
                                   ctypes.byref(o), ctypes.byref(info), _stream(plan.device)))
    return u, info.as_dict(st)


def ddm_solve(plan: Plan, mu, K, alpha, U, f_extra=None, opts=None):
    """Returns (p, u, drag (3,) numpy-like list, info dict)."""
    if f_extra is not None:
        f_extra = _dev(f_extra, (3, plan.n), "f_extra")
    p = torch.empty((plan.n,), dtype=torch.float64, device=plan.device)
    u = torch.empty((3, plan.n), dtype=torch.float64, device=plan.device)
    Uc = (ctypes.c_double * 3)(*[float(v) for v in U])
    drag = (ctypes.c_double * 3)()
    prm, o, info = _params(mu, K, alpha), _opts(opts), Info()
    st = _check(lib().ddm_solve(plan.handle, ctypes.byref(prm), Uc, _ptr(f_extra), _ptr(p), _ptr(u), drag,
                                ctypes.byref(o), ctypes.byref(info), _stream(plan.device)))
    return p, u, [drag[0], drag[1], drag[2]], info.as_dict(st)


def ddm_adjoint(plan: Plan, mu, K, alpha, U, p, u, dJ_ddrag, f_extra=None, opts=None):
    """Gradient of J = dJ_ddrag . drag at the converged ddm_solve outputs (p, u).

    Returns (dJ_dx (3, N) device tensor, dJ_dlogK, dJ_dalpha, info dict).
    """
    p = _dev(p, (plan.n,), "p")
    u = _dev(u, (3, plan.n), "u")
    if f_extra is not None:
        f_extra = _dev(f_extra, (3, plan.n), "f_extra")
    gx = torch.empty((3, plan.n), dtype=torch.float64, device=plan.device)
    Uc = (ctypes.c_double * 3)(*[float(v) for v in U])
    ec = (ctypes.c_double * 3)(*[float(v) for v in dJ_ddrag])
    gK, ga = ctypes.c_double(0.0), ctypes.c_double(0.0)
    prm, o, info = _params(mu, K, alpha), _opts(opts), Info()
    st = _check(lib().ddm_adjoint(plan.handle, ctypes.byref(prm), Uc, _ptr(f_extra), _ptr(p), _ptr(u), ec, _ptr(gx),
                                  ctypes.byref(gK), ctypes.byref(ga), ctypes.byref(o), ctypes.byref(info),
                                  _stream(plan.device)))
    return gx, gK.value, ga.value, info.as_dict(st)


def ddm_dn_spectrum(plan: Plan, mu, K, alpha, v0, m: int, k: int, opts=None):
    """Ritz values of the linear D-N map after m Arnoldi steps from v0 (device (N,)):
    returns (k complex values in decreasing modulus, info dict)."""
    v0 = _dev(v0, (plan.n,), "v0")
    re, im = (ctypes.c_double * k)(), (ctypes.c_double * k)()
    prm, o, info = _params(mu, K, alpha), _opts(opts), Info()
    st = _check(lib().ddm_dn_spectrum(plan.handle, ctypes.byref(prm), _ptr(v0), int(m), int(k), re, im,
                                      ctypes.byref(o), ctypes.byref(info), _stream(plan.device)))
    return [complex(re[i], im[i]) for i in range(k)], info.as_dict(st)


def hessenberg_eigenvalues(H):
    """Eigenvalues (complex list) of the upper Hessenberg matrix H (host, n x n nested sequence or array)."""
    n = len(H)
    flat = (ctypes.c_double * (n * n))(*[float(H[i][j]) for i in range(n) for j in range(n)])
    re, im = (ctypes.c_double * n)(), (ctypes.c_double * n)()
    _check(lib().sdbie_hessenberg_eigenvalues(n, flat, re, im), allow_not_converged=False)
    return [complex(re[i], im[i]) for i in range(n)]
