"""Thin ctypes binding of libmsb (include/msb.h): argument marshalling only.

Every function here forwards to the C entry point of the same name; tensors
are passed as raw device pointers on torch's current stream.  Nothing is
computed in Python.  When libmsb.so is missing, importing the library raises
-- there is no fallback path.

Tensor conventions (complex128, CUDA, contiguous):
  links     (4, 3, 3, V)          U_nu(x)_{ab}
  spinors   (nrhs, 12, V)         k = 3*spin + colour, site x + Lx(y + Ly(z + Lz t))
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  -- loads torch's HIP runtime first; libmsb binds to it

__all__ = [
    "MsbError", "Lattice", "SolveInfo", "Context", "lib", "library_path",
    "neuberger_pfe", "wilson_apply", "mshift_bicgstabl", "mshift_bicgstabl_noalloc", "mshift_cg", "pfe_sign_apply",
    "pfe_sign_backward", "spectral_radius",
    "G5_LEFT", "NEG_MU", "DAGGER", "MIXED", "PERSISTENT", "OVERLAP", "ADJOINT", "REFINE", "DEFERRED", "OP_WILSON",
    "SEED_BASIS",
    "OK", "ERR_ARG", "ERR_HIP", "ERR_OOM", "NOT_CONVERGED", "BREAKDOWN", "REDUCED_ACCURACY", "SUCCESS",
]

OK, ERR_ARG, ERR_HIP, ERR_OOM, NOT_CONVERGED, BREAKDOWN, REDUCED_ACCURACY = 0, 1, 2, 3, 4, 5, 6
# statuses of a completed solve: MSB_OK, and MSB_REDUCED_ACCURACY (mixed
# precision without the per-shift FP64 check); the default `allow` of the
# solver methods (info.status tells them apart)
SUCCESS = (OK, REDUCED_ACCURACY)
G5_LEFT, NEG_MU, DAGGER, MIXED, PERSISTENT, OVERLAP, ADJOINT, REFINE, DEFERRED = 1, 2, 4, 8, 16, 32, 64, 128, 256
OP_WILSON = 512     # A = a D_w instead of a (gamma5 D_w)^2 (multi-mass propagators)
SEED_BASIS = 1024   # passes 2, 3: the seed's lower vectors as coefficients on the iteration's basis

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(_HERE, "_lib", "libmsb.so")


class MsbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[msb status {status}] {msg}")
        self.status = status


class _Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("mass", ctypes.c_double),
                ("mu", ctypes.c_double), ("bc_t", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("bicg_steps", ctypes.c_int), ("mv_count", ctypes.c_longlong),
                ("dot_count", ctypes.c_longlong), ("axpy_count", ctypes.c_longlong),
                ("reliable_updates", ctypes.c_int), ("bytes_model", ctypes.c_double),
                ("shift_iters", ctypes.POINTER(ctypes.c_int)),
                ("shift_resid", ctypes.POINTER(ctypes.c_double)),
                ("shift_true_resid", ctypes.POINTER(ctypes.c_double)),
                ("force_iters", ctypes.POINTER(ctypes.c_int)),
                ("refined_shifts", ctypes.c_int), ("shadow", ctypes.c_void_p),
                ("stored_iters", ctypes.c_int)]


_LIB = None
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
_DP = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load libmsb.so (once)."""
    global _LIB
    if _LIB is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run `python -m paper_1010_2592_amd.build`")
        L = ctypes.CDLL(path)
        L.msb_last_error.restype = ctypes.c_char_p
        L.msb_last_error.argtypes = []
        L.msb_create.argtypes = [ctypes.POINTER(_P), ctypes.POINTER(_Lattice), _P, _P]
        L.msb_destroy.argtypes = [_P]
        L.msb_destroy.restype = None
        L.msb_set_stream.argtypes = [_P, _P]
        L.msb_neuberger_pfe.argtypes = [_I, _DP, _DP]
        L.msb_spectral_radius.argtypes = [_P, _P, _I, _DP]
        L.wilson_apply.argtypes = [_P, _P, _P, _I, _I]
        L.mshift_bicgstabl.argtypes = [_P, _D, _I, _DP, _DP, _I, _I, _D, _I, _I, _I, _I,
                                       _P, _P, _P, ctypes.POINTER(_Info)]
        L.mshift_bicgstabl_noalloc.argtypes = L.mshift_bicgstabl.argtypes
        L.mshift_cg.argtypes = [_P, _D, _I, _DP, _DP, _I, _D, _I, _I, _I, _I, _P, _P, _P,
                                ctypes.POINTER(_Info)]
        L.pfe_sign_apply.argtypes = [_P, _D, _I, _DP, _DP, _I, _D, _I, _I, _I, _I, _P, _P,
                                     ctypes.POINTER(_Info)]
        L.msb_low_modes.argtypes = [_P, _I, _I, _P, _D, _I, _I, _DP, _P, _DP, ctypes.POINTER(_I)]
        L.pfe_sign_apply_deflated.argtypes = [_P, _D, _I, _DP, _DP, _I, _D, _I, _I, _I, _I, _I, _DP, _P,
                                              _P, _P, ctypes.POINTER(_Info)]
        L.pfe_sign_backward.argtypes = [_P, _D, _I, _DP, _DP, _I, _D, _I, _I, _I, _P, _P, _I,
                                        _P, _DP, _DP, _P, ctypes.POINTER(_Info)]
        L.msb_set_store_limit.argtypes = [_P, ctypes.c_ulonglong]
        L.msb_profile_enable.argtypes = [_P, _I]
        L.msb_profile_classes.argtypes = [_P, ctypes.c_uint, _I]
        L.msb_profile_read.argtypes = [_P, _I, ctypes.POINTER(ctypes.c_longlong), _DP, _DP]
        for f in ("msb_create", "msb_set_stream", "msb_neuberger_pfe", "msb_spectral_radius",
                  "msb_set_store_limit", "msb_profile_enable", "msb_profile_classes", "msb_profile_read",
                  "wilson_apply", "mshift_bicgstabl", "mshift_bicgstabl_noalloc", "mshift_cg", "pfe_sign_apply", "pfe_sign_backward",
                  "msb_low_modes", "pfe_sign_apply_deflated"):
            getattr(L, f).restype = _I
        _LIB = L
    return _LIB


def _check(rc: int, allow=SUCCESS):
    if rc not in allow:
        raise MsbError(rc, lib().msb_last_error().decode())
    return rc


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _spinors(t: torch.Tensor, V: int, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3 or t.shape[1] != 12 or t.shape[2] != V:
        raise ValueError(f"{name} must have shape (nrhs, 12, {V})")
    return t.contiguous()


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Lattice:
    dims: Sequence[int]
    mass: float = -2.0
    mu: float = 0.0
    bc_t: int = -1

    @property
    def volume(self) -> int:
        return int(np.prod(self.dims))


@dataclass
class SolveInfo:
    status: int
    outer_iters: int
    bicg_steps: int
    mv_count: int
    dot_count: int
    axpy_count: int
    reliable_updates: int
    bytes_model: float
    shift_iters: np.ndarray
    shift_resid: np.ndarray
    shift_true_resid: Optional[np.ndarray]
    refined_shifts: int = 0
    stored_iters: int = -1


def neuberger_pfe(n: int):
    """(sigma, w) of the n-pole Neuberger expansion, from the library."""
    s = np.zeros(n)
    w = np.zeros(n)
    _check(lib().msb_neuberger_pfe(int(n), _dptr(s), _dptr(w)))
    return s, w


class Context:
    """An msb_ctx: lattice geometry, D_w(mu) parameters and a copy of the links."""

    def __init__(self, lat: Lattice, links: torch.Tensor):
        V = lat.volume
        if links.dtype != torch.complex128 or not links.is_cuda or tuple(links.shape) != (4, 3, 3, V):
            raise ValueError(f"links must be a complex128 CUDA tensor of shape (4, 3, 3, {V})")
        links = links.contiguous()
        self.lat = lat
        self.V = V
        cl = _Lattice((ctypes.c_int * 4)(*[int(d) for d in lat.dims]), float(lat.mass),
                      float(lat.mu), int(lat.bc_t))
        h = _P()
        _check(lib().msb_create(ctypes.byref(h), ctypes.byref(cl), _P(links.data_ptr()),
                                _stream_handle()))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().msb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_store_limit(self, nbytes: int):
        """Bytes the pseudo-double pass may keep in its store (0: no limit)."""
        _check(lib().msb_set_store_limit(self._h, int(nbytes)))

    def _sync_stream(self):
        _check(lib().msb_set_stream(self._h, _stream_handle()))

    # -- kernel timing ------------------------------------------------------
    PROFILE_CLASSES = ("stencil", "shift_update", "shift_mr_update", "seed_vector", "scalar", "other")

    def profile_enable(self, on: bool = True, classes=None, stride: int = 1):
        """Record kernel timings from now on (on=False stops); classes: the
        names of PROFILE_CLASSES to record, None for all; stride: every
        stride-th of those launches."""
        self._sync_stream()
        mask = 0xFFFFFFFF
        if classes is not None:
            mask = 0
            for k in classes:
                mask |= 1 << self.PROFILE_CLASSES.index(k)
        _check(lib().msb_profile_classes(self._h, mask, int(stride)))
        _check(lib().msb_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        n = len(self.PROFILE_CLASSES)
        cnt = (ctypes.c_longlong * n)()
        ms = np.zeros(n)
        by = np.zeros(n)
        _check(lib().msb_profile_read(self._h, n, cnt, _dptr(ms), _dptr(by)))
        return {k: {"count": int(cnt[i]), "ms": float(ms[i]), "bytes": float(by[i])}
                for i, k in enumerate(self.PROFILE_CLASSES)}

    # -- entry points ------------------------------------------------------
    def wilson_apply(self, x: torch.Tensor, flags: int = 0, out: Optional[torch.Tensor] = None):
        x = _spinors(x, self.V, "in")
        if out is None:
            out = torch.empty_like(x)
        self._sync_stream()
        _check(lib().wilson_apply(self._h, _P(x.data_ptr()), _P(out.data_ptr()), x.shape[0], int(flags)))
        return out

    def spectral_radius(self, start: torch.Tensor, iters: int = 100) -> float:
        start = _spinors(start, self.V, "start")
        rho = ctypes.c_double(0.0)
        self._sync_stream()
        _check(lib().msb_spectral_radius(self._h, _P(start.data_ptr()), int(iters), ctypes.byref(rho)))
        return rho.value

    def _info(self, nrhs, ns, force_iters, true_resid):
        info = _Info()
        it = np.zeros(nrhs * ns, dtype=np.int32)
        rs = np.zeros(nrhs * ns)
        tr = np.zeros(nrhs * ns) if true_resid else None
        info.shift_iters = it.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        info.shift_resid = _dptr(rs)
        info.shift_true_resid = _dptr(tr) if tr is not None else ctypes.POINTER(ctypes.c_double)()
        fi = None
        if force_iters is not None:
            fi = np.ascontiguousarray(np.broadcast_to(np.asarray(force_iters, dtype=np.int32),
                                                      (nrhs, ns)).reshape(-1))
            info.force_iters = fi.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        return info, (it, rs, tr, fi)

    @staticmethod
    def _pack_info(info, keep, nrhs, ns):
        it, rs, tr, _ = keep
        return SolveInfo(info.status, info.outer_iters, info.bicg_steps, info.mv_count,
                         info.dot_count, info.axpy_count, info.reliable_updates, info.bytes_model,
                         it.reshape(nrhs, ns).copy(), rs.reshape(nrhs, ns).copy(),
                         None if tr is None else tr.reshape(nrhs, ns).copy(), info.refined_shifts,
                         info.stored_iters)

    def mshift_bicgstabl(self, b: torch.Tensor, a_scale: float, shifts, weights, l: int,
                         tol: float, max_outer: int, pass_: int = 1, flags: int = 0,
                         want_shifts: bool = False, force_iters=None, true_resid: bool = False,
                         allow=SUCCESS, shadow: Optional[torch.Tensor] = None, y: Optional[torch.Tensor] = None):
        """y = sum_s w_s (A + sigma_s)^{-1} b; returns (y, info, x_shifts or None).

        shifts/weights: (n_shift,) for one set, or (nrhs, n_shift) per rhs.
        pass_: 1 single pass, 2 double pass, 3 pseudo-double pass (the Mv
        outputs of the first pass kept in device memory and summed after the
        sweep).  shadow: optional shadow residual r~ of BiCGstab(l) (default
        b; a random r~ for point sources under OP_WILSON).  y: optional
        output tensor (written)."""
        return self._mshift("mshift_bicgstabl", b, a_scale, shifts, weights, l, tol, max_outer, pass_, flags,
                            want_shifts, force_iters, true_resid, allow, shadow, y)

    def mshift_bicgstabl_noalloc(self, b: torch.Tensor, a_scale: float, shifts, weights, l: int,
                                 tol: float, max_outer: int, pass_: int = 1, flags: int = 0,
                                 want_shifts: bool = False, force_iters=None, true_resid: bool = False,
                                 allow=SUCCESS, shadow: Optional[torch.Tensor] = None,
                                 y: Optional[torch.Tensor] = None, x_shifts: Optional[torch.Tensor] = None):
        """mshift_bicgstabl with the library's workspace taken from its fixed
        device scratch array (no device allocation in the call); pass_ 1 or 2.
        Pass y (and x_shifts) to keep this call itself free of allocations."""
        return self._mshift("mshift_bicgstabl_noalloc", b, a_scale, shifts, weights, l, tol, max_outer, pass_,
                            flags, want_shifts, force_iters, true_resid, allow, shadow, y, x_shifts)

    def _mshift(self, fn, b, a_scale, shifts, weights, l, tol, max_outer, pass_, flags, want_shifts,
                force_iters, true_resid, allow, shadow, y=None, x_shifts=None):
        b = _spinors(b, self.V, "b")
        nrhs = b.shape[0]
        sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64))
        wt = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        per = 1 if sh.ndim == 2 else 0
        ns = sh.shape[-1]
        if y is None:
            y = torch.empty_like(b)
        elif y.shape != b.shape or y.dtype != b.dtype or y.device != b.device or not y.is_contiguous():
            raise ValueError("y must be a contiguous tensor of b's shape, dtype and device")
        xs = x_shifts
        if xs is None and want_shifts:
            xs = torch.zeros((nrhs, ns, 12, self.V), dtype=torch.complex128, device=b.device)
        if xs is not None and (tuple(xs.shape) != (nrhs, ns, 12, self.V) or xs.dtype != torch.complex128
                               or xs.device != b.device or not xs.is_contiguous()):
            raise ValueError(f"x_shifts must be a contiguous complex128 tensor of shape ({nrhs}, {ns}, 12, {self.V})")
        info, keep = self._info(nrhs, ns, force_iters, true_resid or bool(flags & REFINE))
        if shadow is not None:
            shadow = _spinors(shadow, self.V, "shadow")
            if shadow.shape != b.shape or shadow.device != b.device:
                raise ValueError("shadow must have the shape and device of b")
            info.shadow = shadow.data_ptr()     # shadow (a local) outlives the call
        self._sync_stream()
        rc = getattr(lib(), fn)(self._h, float(a_scale), ns, _dptr(sh), _dptr(wt), per, int(l),
                                    float(tol), int(max_outer), int(pass_), int(flags), nrhs,
                                    _P(b.data_ptr()), _P(y.data_ptr()),
                                    _P(xs.data_ptr() if xs is not None else None), ctypes.byref(info))
        _check(rc, allow)
        return y, self._pack_info(info, keep, nrhs, ns), xs

    def mshift_cg(self, b: torch.Tensor, a_scale: float, shifts, weights, tol: float, max_iter: int,
                  pass_: int = 1, want_shifts: bool = False, force_iters=None, allow=SUCCESS):
        """Multi-shift CG (the context must have mu = 0): y = sum_s w_s (A + sigma_s)^{-1} b;
        returns (y, info, x_shifts or None).  pass_: 1 single, 2 double, 3 pseudo-double."""
        b = _spinors(b, self.V, "b")
        nrhs = b.shape[0]
        sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64))
        wt = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        per = 1 if sh.ndim == 2 else 0
        ns = sh.shape[-1]
        y = torch.empty_like(b)
        xs = torch.zeros((nrhs, ns, 12, self.V), dtype=torch.complex128, device=b.device) \
            if want_shifts else None
        info, keep = self._info(nrhs, ns, force_iters, False)
        self._sync_stream()
        rc = lib().mshift_cg(self._h, float(a_scale), ns, _dptr(sh), _dptr(wt), per, float(tol), int(max_iter),
                             int(pass_), 0, nrhs, _P(b.data_ptr()), _P(y.data_ptr()),
                             _P(xs.data_ptr() if xs is not None else None), ctypes.byref(info))
        _check(rc, allow)
        return y, self._pack_info(info, keep, nrhs, ns), xs

    def low_modes(self, nev: int, start: torch.Tensor, tol: float = 1e-10, degree: int = 24,
                  max_iter: int = 200, allow=SUCCESS):
        """Low modes of H = gamma5 D_w (mu = 0): (evals [nev] sorted by |lambda|,
        evecs [nev][12][V], resid [nev], iterations).  start: [nblock][12][V]
        complex128 start block, nblock > nev."""
        start = _spinors(start, self.V, "start")
        ev = np.zeros(nev)
        rs = np.zeros(nev)
        it = ctypes.c_int(0)
        evecs = torch.empty((nev, 12, self.V), dtype=torch.complex128, device=start.device)
        self._sync_stream()
        rc = lib().msb_low_modes(self._h, int(nev), start.shape[0], _P(start.data_ptr()), float(tol), int(degree),
                                 int(max_iter), _dptr(ev), _P(evecs.data_ptr()), _dptr(rs), ctypes.byref(it))
        _check(rc, allow)
        return ev, evecs, rs, it.value

    def pfe_sign_apply_deflated(self, b: torch.Tensor, a_scale: float, shifts, weights, l: int, tol: float,
                                max_outer: int, evals, evecs: torch.Tensor, pass_: int = 1, flags: int = 0,
                                allow=SUCCESS):
        """sign(H) b (or the overlap with OVERLAP) with the low modes (evals,
        evecs) deflated; mu = 0."""
        b = _spinors(b, self.V, "b")
        evecs = _spinors(evecs, self.V, "evecs")
        nrhs = b.shape[0]
        ev = np.ascontiguousarray(np.asarray(evals, dtype=np.float64))
        sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64))
        wt = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        ns = sh.shape[-1]
        out = torch.empty_like(b)
        info, keep = self._info(nrhs, ns, None, False)
        self._sync_stream()
        rc = lib().pfe_sign_apply_deflated(self._h, float(a_scale), ns, _dptr(sh), _dptr(wt), int(l), float(tol),
                                           int(max_outer), int(pass_), int(flags), nrhs, len(ev), _dptr(ev),
                                           _P(evecs.data_ptr()), _P(b.data_ptr()), _P(out.data_ptr()),
                                           ctypes.byref(info))
        _check(rc, allow)
        return out, self._pack_info(info, keep, nrhs, ns)

    def pfe_sign_apply(self, b: torch.Tensor, a_scale: float, shifts, weights, l: int, tol: float,
                       max_outer: int, pass_: int = 1, flags: int = 0, force_iters=None,
                       allow=SUCCESS):
        b = _spinors(b, self.V, "b")
        nrhs = b.shape[0]
        sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64))
        wt = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        ns = sh.shape[-1]
        out = torch.empty_like(b)
        info, keep = self._info(nrhs, ns, force_iters, False)
        self._sync_stream()
        rc = lib().pfe_sign_apply(self._h, float(a_scale), ns, _dptr(sh), _dptr(wt), int(l), float(tol),
                                  int(max_outer), int(pass_), int(flags), nrhs, _P(b.data_ptr()),
                                  _P(out.data_ptr()), ctypes.byref(info))
        _check(rc, allow)
        return out, self._pack_info(info, keep, nrhs, ns)

    def pfe_sign_backward(self, b: torch.Tensor, eta: torch.Tensor, a_scale: float, shifts, weights,
                          l: int, tol: float, max_outer: int, mode: int = 0, flags: int = 0,
                          grad_links: Optional[torch.Tensor] = None, force_iters=None, allow=SUCCESS):
        """Gradients of Re<eta, y>, y = f(A) b (mode 0) or sign(H) b (mode 1).

        Returns (grad_b, grad_w, grad_sigma, grad_links, info); grad_links is
        accumulated into the given tensor (or a fresh zero tensor)."""
        b = _spinors(b, self.V, "b")
        eta = _spinors(eta, self.V, "eta")
        nrhs = b.shape[0]
        sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64))
        wt = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        ns = sh.shape[-1]
        gb = torch.empty_like(b)
        gw = np.zeros(ns)
        gs = np.zeros(ns)
        if grad_links is None:
            grad_links = torch.zeros((4, 3, 3, self.V), dtype=torch.complex128, device=b.device)
        info, keep = self._info(nrhs, ns, force_iters, False)
        self._sync_stream()
        rc = lib().pfe_sign_backward(self._h, float(a_scale), ns, _dptr(sh), _dptr(wt), int(l),
                                     float(tol), int(max_outer), int(flags), nrhs, _P(b.data_ptr()),
                                     _P(eta.data_ptr()), int(mode), _P(gb.data_ptr()), _dptr(gw),
                                     _dptr(gs), _P(grad_links.data_ptr()), ctypes.byref(info))
        _check(rc, allow)
        return gb, gw, gs, grad_links, self._pack_info(info, keep, nrhs, ns)


# module-level forms with the C names (first argument: the Context)
def wilson_apply(ctx: Context, x, flags=0, out=None):
    return ctx.wilson_apply(x, flags, out)


def spectral_radius(ctx: Context, start, iters=100):
    return ctx.spectral_radius(start, iters)


def mshift_bicgstabl(ctx: Context, b, a_scale, shifts, weights, l, tol, max_outer, pass_=1, **kw):
    return ctx.mshift_bicgstabl(b, a_scale, shifts, weights, l, tol, max_outer, pass_, **kw)


def mshift_bicgstabl_noalloc(ctx: Context, b, a_scale, shifts, weights, l, tol, max_outer, pass_=1, **kw):
    return ctx.mshift_bicgstabl_noalloc(b, a_scale, shifts, weights, l, tol, max_outer, pass_, **kw)


def mshift_cg(ctx: Context, b, a_scale, shifts, weights, tol, max_iter, pass_=1, **kw):
    return ctx.mshift_cg(b, a_scale, shifts, weights, tol, max_iter, pass_, **kw)


def pfe_sign_apply(ctx: Context, b, a_scale, shifts, weights, l, tol, max_outer, pass_=1, **kw):
    return ctx.pfe_sign_apply(b, a_scale, shifts, weights, l, tol, max_outer, pass_, **kw)


def pfe_sign_backward(ctx: Context, b, eta, a_scale, shifts, weights, l, tol, max_outer, **kw):
    return ctx.pfe_sign_backward(b, eta, a_scale, shifts, weights, l, tol, max_outer, **kw)
