"""Python binding of libmgfr.so (include/mgfr.h): argument marshalling only.

Every step of the solve runs in the HIP library; PyTorch supplies device memory and the
stream.  The names follow the C ABI: mgfr_create, mg_fr_solve, mgfr_residual, ...  Loading
fails loudly when the library has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field, fields

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgfr.so")

MGFR_OK, MGFR_EINVAL, MGFR_ENONFINITE, MGFR_ENOTCONV, MGFR_EDEVICE, MGFR_ENOMEM = 0, -1, -2, -3, -4, -5
MGFR_FP64, MGFR_MIXED = 0, 1
MGFR_SUBTRACT_MEAN, MGFR_WARM_START, MGFR_PROFILE, MGFR_GRAPH, MGFR_PER_PHASE = 1, 2, 4, 8, 16
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENONFINITE", -3: "ENOTCONV", -4: "EDEVICE", -5: "ENOMEM"}


class mgfr_params(ctypes.Structure):
    _fields_ = [("omega_m", ctypes.c_double), ("omega_l", ctypes.c_double), ("a", ctypes.c_double),
                ("n", ctypes.c_double), ("fr0_abs", ctypes.c_double), ("box_mpc_h", ctypes.c_double)]


class mgfr_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("pre", ctypes.c_int), ("post", ctypes.c_int),
                ("coarsest_n", ctypes.c_int), ("coarsest_sweeps", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("precision", ctypes.c_int), ("flags", ctypes.c_int),
                ("inner_cycles", ctypes.c_int), ("max_step", ctypes.c_double),
                ("coarsest_rtol", ctypes.c_double), ("planes", ctypes.c_int), ("tau_alpha", ctypes.c_double),
                ("unit_n", ctypes.c_int), ("tile", ctypes.c_int)]


class mgfr_patch(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("parent", ctypes.c_int), ("origin", ctypes.c_int * 3),
                ("n", ctypes.c_int), ("offset", ctypes.c_longlong)]


class mgfr_stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("inner_cycles", ctypes.c_int),
                ("cell_updates", ctypes.c_longlong), ("finest_updates", ctypes.c_longlong),
                ("sweep_launches", ctypes.c_int), ("sweep_ms", ctypes.c_double),
                ("sweep_bytes", ctypes.c_double), ("solve_ms", ctypes.c_double), ("tau_rms", ctypes.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


@dataclass
class Params:
    """Hu-Sawicki f(R) model and box (mirrors mgfr_params)."""
    omega_m: float = 0.24
    omega_l: float = -1.0
    a: float = 1.0
    n: float = 1.0
    fr0_abs: float = 1e-5
    box_mpc_h: float = 64.0

    def c(self) -> mgfr_params:
        return mgfr_params(*[getattr(self, f.name) for f in fields(self)])


_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """The loaded libmgfr.so (raises LibraryMissing if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        P, O = ctypes.POINTER(mgfr_params), ctypes.POINTER(mgfr_opts)
        sig = {
            "mgfr_create": ([ctypes.POINTER(vp), ctypes.c_int], ctypes.c_int),
            "mgfr_destroy": ([vp], None),
            "mgfr_last_error": ([vp], ctypes.c_char_p),
            "mgfr_default_opts": ([O], None),
            "mgfr_get_stats": ([vp, ctypes.POINTER(mgfr_stats)], ctypes.c_int),
            "mgfr_constants": ([P, ctypes.c_int, dp], ctypes.c_int),
            "mgfr_residual": ([vp, vp, vp, ctypes.c_int, P, ctypes.c_int, vp, vp], ctypes.c_int),
            "mg_fr_solve": ([vp, vp, ctypes.c_int, P, O, vp, dp, ip, vp], ctypes.c_int),
            "mg_fr_solve_noalloc": ([vp, vp, ctypes.c_int, P, O, vp, dp, ip, vp], ctypes.c_int),
            "mgfr_smooth": ([vp, vp, vp, ctypes.c_int, P, O, ctypes.c_int, ctypes.c_int, vp], ctypes.c_int),
            "mgfr_smooth32": ([vp, vp, vp, vp, ctypes.c_int, P, O, ctypes.c_int, ctypes.c_int, vp], ctypes.c_int),
            "mg_fr_solve_patches": ([vp, vp, ctypes.c_int, ctypes.POINTER(mgfr_patch), ctypes.c_int, vp, vp,
                                     ctypes.c_longlong, P, O, dp, ip, vp], ctypes.c_int),
            "mg_fr_solve_batch": ([vp, ctypes.c_int, ip, ctypes.POINTER(vp), P, O, ctypes.POINTER(vp), dp, ip, vp],
                                  ctypes.c_int),
            "mgfr_autotune": ([vp, vp, ctypes.c_int, P, O, vp, O, dp, vp], ctypes.c_int),
            "mg_poisson_solve": ([vp, vp, vp, ctypes.c_int, P, O, vp, dp, ip, vp], ctypes.c_int),
            "mgfr_tau": ([vp, vp, vp, ctypes.c_int, P, ctypes.c_int, vp, dp, vp], ctypes.c_int),
            "mg_poisson_smooth": ([vp, vp, vp, ctypes.c_int, P, ctypes.c_int, ctypes.c_int, vp, vp], ctypes.c_int),
            "mg_fr_solve_masked": ([vp, vp, vp, ctypes.c_int, P, O, vp, dp, ip, vp], ctypes.c_int),
            "mgfr_tsc_density": ([vp, vp, ctypes.c_longlong, ctypes.c_int, ctypes.c_double, vp, vp], ctypes.c_int),
            "mgfr_tsc_force": ([vp, vp, ctypes.c_int, vp, ctypes.c_longlong, vp, vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return ("mgfr_create", "mgfr_destroy", "mgfr_last_error", "mgfr_default_opts", "mgfr_constants",
            "mgfr_residual", "mg_fr_solve", "mg_fr_solve_noalloc", "mgfr_get_stats", "mgfr_smooth", "mgfr_smooth32", "mg_fr_solve_patches",
            "mg_fr_solve_batch", "mgfr_autotune", "mg_poisson_solve", "mg_poisson_smooth", "mgfr_tau",
            "mg_fr_solve_masked", "mgfr_tsc_density", "mgfr_tsc_force")


def mgfr_default_opts(**overrides) -> mgfr_opts:
    o = mgfr_opts()
    lib().mgfr_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(f"mgfr_opts has no field {k}")
        setattr(o, k, v)
    return o


CONST_NAMES = ("xi", "ctilde", "K", "A", "Sbar", "D", "ubar", "C")


def mgfr_constants(params: Params, N: int) -> dict:
    out = (ctypes.c_double * 8)()
    st = lib().mgfr_constants(ctypes.byref(params.c()), N, out)
    if st != MGFR_OK:
        raise ValueError(f"mgfr_constants failed ({STATUS_NAMES.get(st, st)})")
    return dict(zip(CONST_NAMES, list(out)))


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class MgfrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Context:
    """Owns an mgfr_ctx on one device (its multigrid scratch persists between calls)."""

    def __init__(self, device: int = 0):
        self.device = device
        h = ctypes.c_void_p()
        st = lib().mgfr_create(ctypes.byref(h), device)
        if st != MGFR_OK:
            raise MgfrError(st, f"mgfr_create(device={device}) failed")
        self.handle = h

    def close(self):
        if self.handle:
            lib().mgfr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().mgfr_last_error(self.handle).decode()


def mgfr_get_stats(ctx: Context) -> dict:
    s = mgfr_stats()
    st = lib().mgfr_get_stats(ctx.handle, ctypes.byref(s))
    if st != MGFR_OK:
        raise MgfrError(st, "mgfr_get_stats failed")
    return s.as_dict()


def mgfr_create(device: int = 0) -> Context:
    return Context(device)


def mgfr_residual(ctx: Context, rho, u, params: Params, flags: int = 0, out=None, stream=None):
    """d = L(u) on the periodic grid (device tensors, float64, N^3)."""
    import torch
    N = rho.shape[0]
    if out is None:
        out = torch.empty_like(u)
    st = lib().mgfr_residual(ctx.handle, _ptr(rho), _ptr(u), N, ctypes.byref(params.c()), flags,
                             _ptr(out), _stream(stream))
    if st != MGFR_OK:
        raise MgfrError(st, ctx.last_error())
    return out


def mgfr_smooth(ctx: Context, rho, u, params: Params, nsweeps: int, variant: int = 0,
                opts: mgfr_opts | None = None, stream=None):
    """nsweeps single-grid red-black Newton-Gauss-Seidel sweeps, in place on u.
    variant 0: solver's choice, 1: per-colour kernels, 2: fused red-black kernel."""
    N = rho.shape[0]
    if opts is None:
        opts = mgfr_default_opts()
    st = lib().mgfr_smooth(ctx.handle, _ptr(rho), _ptr(u), N, ctypes.byref(params.c()), ctypes.byref(opts),
                           nsweeps, variant, _stream(stream))
    if st != MGFR_OK:
        raise MgfrError(st, ctx.last_error())
    return u


def mgfr_smooth32(ctx: Context, ub, e, f, params: Params, nsweeps: int, variant: int = 0,
                  opts: mgfr_opts | None = None, stream=None):
    """nsweeps red-black Newton-Gauss-Seidel sweeps of the single-precision correction
    equation N(e) = f about the base ub (float32 device tensors of shape (N, N, N)), in place
    on e.  variant 0: the mixed solver's finest-level kernel, 1: per-colour kernels, 2: fused
    red-black kernel (opts.planes planes per workgroup, 0 = automatic)."""
    import torch
    for t in (ub, e, f):
        if t.dtype != torch.float32:
            raise TypeError("ub, e and f must be float32")
    N = ub.shape[0]
    if opts is None:
        opts = mgfr_default_opts()
    st = lib().mgfr_smooth32(ctx.handle, _ptr(ub), _ptr(e), _ptr(f), N, ctypes.byref(params.c()),
                             ctypes.byref(opts), nsweeps, variant, _stream(stream))
    if st != MGFR_OK:
        raise MgfrError(st, ctx.last_error())
    return e


def mg_fr_solve(ctx: Context, rho, params: Params, opts: mgfr_opts | None = None, u=None,
                stream=None, raise_on_error: bool = True):
    """Solves the domain grid.  rho, u: float64 device tensors of shape (N, N, N); u is
    written in place (and read as the start field with MGFR_WARM_START).
    Returns (u, residual history as a numpy array, status)."""
    import torch
    N = rho.shape[0]
    if opts is None:
        opts = mgfr_default_opts()
    if u is None:
        u = torch.empty_like(rho)
    hist = np.zeros(opts.max_cycles + 1)
    nh = ctypes.c_int(0)
    st = lib().mg_fr_solve(ctx.handle, _ptr(rho), N, ctypes.byref(params.c()), ctypes.byref(opts), _ptr(u),
                           hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(nh),
                           _stream(stream))
    if raise_on_error and st not in (MGFR_OK, MGFR_ENOTCONV):
        raise MgfrError(st, ctx.last_error())
    return u, hist[:nh.value].copy(), st


def mg_fr_solve_noalloc(ctx: Context, rho, u, params: Params, opts: mgfr_opts | None = None, stream=None,
                        raise_on_error: bool = True):
    """mg_fr_solve with every scratch buffer in the library's fixed device array (N <= 128):
    nothing is allocated by the call.  rho, u: float64 device tensors of shape (N, N, N); u is
    written in place.  Returns (u, residual history, status)."""
    N = rho.shape[0]
    if opts is None:
        opts = mgfr_default_opts()
    hist = np.zeros(opts.max_cycles + 1)
    nh = ctypes.c_int(0)
    st = lib().mg_fr_solve_noalloc(ctx.handle, _ptr(rho), N, ctypes.byref(params.c()), ctypes.byref(opts),
                                   _ptr(u), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(nh), _stream(stream))
    if raise_on_error and st not in (MGFR_OK, MGFR_ENOTCONV):
        raise MgfrError(st, ctx.last_error())
    return u, hist[:nh.value].copy(), st


def mgfr_tau(ctx: Context, rho, u, params: Params, flags: int = 0, stream=None):
    """Truncation-error estimate tau = L^H(R u) - R L^h(u) of the field u (float64 device
    tensors of shape (N, N, N)).  Returns (tau on the (N/2)^3 level, rms of tau)."""
    import torch
    N = rho.shape[0]
    tau = torch.empty((N // 2,) * 3, dtype=torch.float64, device=rho.device)
    r = ctypes.c_double(0.0)
    st = lib().mgfr_tau(ctx.handle, _ptr(rho), _ptr(u), N, ctypes.byref(params.c()), flags, _ptr(tau),
                        ctypes.byref(r), _stream(stream))
    if st != MGFR_OK:
        raise MgfrError(st, ctx.last_error())
    return tau, r.value


def mg_fr_solve_masked(ctx: Context, rho, mask, u, params: Params, opts: mgfr_opts | None = None, stream=None,
                       raise_on_error: bool = True):
    """Refinement level with the mask scheme.  rho, u: float64 device tensors (N, N, N); mask:
    float32 device tensor (N, N, N) in [-1, 1], active where > 0; u holds the initial guess in
    active cells and the fixed values elsewhere and is solved in place.
    Returns (u, residual history over the active cells, status)."""
    import torch
    if rho.dtype != torch.float64 or u.dtype != torch.float64 or mask.dtype != torch.float32:
        raise TypeError("rho and u must be float64 and mask float32")
    N = rho.shape[0]
    if tuple(rho.shape) != (N,) * 3 or tuple(mask.shape) != (N,) * 3 or tuple(u.shape) != (N,) * 3:
        raise ValueError("rho, mask and u must all have shape (N, N, N)")
    if opts is None:
        opts = mgfr_default_opts()
    hist = np.zeros(opts.max_cycles + 1)
    nh = ctypes.c_int(0)
    st = lib().mg_fr_solve_masked(ctx.handle, _ptr(rho), _ptr(mask), N, ctypes.byref(params.c()), ctypes.byref(opts),
                                  _ptr(u), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(nh),
                                  _stream(stream))
    if raise_on_error and st not in (MGFR_OK, MGFR_ENOTCONV):
        raise MgfrError(st, ctx.last_error())
    return u, hist[:nh.value].copy(), st


def mgfr_tsc_density(ctx: Context, pos, N: int, mass: float, rho=None, stream=None):
    """TSC density of particles pos (float64 device tensor (np, 3), box units) on the N^3 grid."""
    import torch
    if pos.dtype != torch.float64 or pos.dim() != 2 or pos.shape[1] != 3:
        raise TypeError("pos must be a float64 (np, 3) tensor")
    if rho is None:
        rho = torch.empty((N,) * 3, dtype=torch.float64, device=pos.device)
    st = lib().mgfr_tsc_density(ctx.handle, _ptr(pos), pos.shape[0], N, float(mass), _ptr(rho), _stream(stream))
    if st != MGFR_OK:
        raise MgfrError(st, ctx.last_error())
    return rho


def mgfr_tsc_force(ctx: Context, phi, pos, acc=None, stream=None):
    """-grad phi interpolated to the particles with the TSC weights: float64 (np, 3)."""
    import torch
    if pos.dtype != torch.float64 or pos.dim() != 2 or pos.shape[1] != 3 or phi.dtype != torch.float64:
        raise TypeError("phi must be float64 and pos a float64 (np, 3) tensor")
    if acc is None:
        acc = torch.empty_like(pos)
    st = lib().mgfr_tsc_force(ctx.handle, _ptr(phi), phi.shape[0], _ptr(pos), pos.shape[0], _ptr(acc),
                              _stream(stream))
    if st != MGFR_OK:
        raise MgfrError(st, ctx.last_error())
    return acc


def mg_poisson_smooth(ctx: Context, rho, u, phi, params: Params, nsweeps: int, variant: int = 0, stream=None):
    """nsweeps single-grid red-black sweeps of the modified Poisson equation, in place on phi
    (float64 device tensors of shape (N, N, N)).  variant 0: per-colour kernels, 1: one-sweep
    fused kernel, 2: two-sweep fused kernel (nsweeps even; N >= 256 for 1 and 2)."""
    N = rho.shape[0]
    st = lib().mg_poisson_smooth(ctx.handle, _ptr(rho), _ptr(u), N, ctypes.byref(params.c()), nsweeps, variant,
                                 _ptr(phi), _stream(stream))
    if st != MGFR_OK:
        raise MgfrError(st, ctx.last_error())
    return phi


def mg_poisson_solve(ctx: Context, rho, u, params: Params, opts: mgfr_opts | None = None, phi=None,
                     stream=None, raise_on_error: bool = True):
    """The modified Poisson equation for the potential phi, given the density rho and the
    scalaron u (float64 device tensors of shape (N, N, N)); opts.tol is relative to the rms of
    the source.  Returns (phi, residual history as a numpy array, status)."""
    import torch
    N = rho.shape[0]
    if opts is None:
        opts = mgfr_default_opts()
    if phi is None:
        phi = torch.empty_like(rho)
    hist = np.zeros(opts.max_cycles + 1)
    nh = ctypes.c_int(0)
    st = lib().mg_poisson_solve(ctx.handle, _ptr(rho), _ptr(u), N, ctypes.byref(params.c()), ctypes.byref(opts),
                                _ptr(phi), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(nh),
                                _stream(stream))
    if raise_on_error and st not in (MGFR_OK, MGFR_ENOTCONV):
        raise MgfrError(st, ctx.last_error())
    return phi, hist[:nh.value].copy(), st


def mg_fr_solve_patches(ctx: Context, u_domain, patches, rho_packed, params: Params,
                        opts: mgfr_opts | None = None, u_packed=None, stream=None, raise_on_error: bool = True):
    """Refinement patches, level by level.  patches: list of dicts {level, parent, origin, n,
    offset}; rho_packed / u_packed: float64 device tensors holding every patch's n^3 block at
    its offset; u_domain: the solved (N0, N0, N0) domain grid.
    Returns (u_packed, per-patch residual histories, status)."""
    import torch
    if opts is None:
        opts = mgfr_default_opts()
    npatch = len(patches)
    arr = (mgfr_patch * max(npatch, 1))()
    for i, p in enumerate(patches):
        arr[i].level = int(p["level"])
        arr[i].parent = int(p["parent"])
        for d in range(3):
            arr[i].origin[d] = int(p["origin"][d])
        arr[i].n = int(p["n"])
        arr[i].offset = int(p["offset"])
    if u_packed is None:
        u_packed = torch.empty_like(rho_packed)
    H = opts.max_cycles + 1
    hist = np.zeros(max(npatch, 1) * H)
    nh = np.zeros(max(npatch, 1), dtype=np.int32)
    st = lib().mg_fr_solve_patches(ctx.handle, _ptr(u_domain), u_domain.shape[0], arr, npatch, _ptr(rho_packed),
                                   _ptr(u_packed), rho_packed.numel(), ctypes.byref(params.c()),
                                   ctypes.byref(opts), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   nh.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _stream(stream))
    if raise_on_error and st not in (MGFR_OK, MGFR_ENOTCONV):
        raise MgfrError(st, ctx.last_error())
    hists = [hist[i * H:i * H + nh[i]].copy() for i in range(npatch)]
    return u_packed, hists, st


def mg_fr_solve_batch(ctx: Context, rhos, params_list, opts: mgfr_opts | None = None, us=None, stream=None,
                      raise_on_error: bool = True):
    """Independent periodic boxes solved together.  rhos: list of (N, N, N) float64 device
    tensors; params_list: one Params per box.  Returns (list of u, histories, status)."""
    import torch
    if opts is None:
        opts = mgfr_default_opts()
    nbox = len(rhos)
    if us is None:
        us = [torch.empty_like(r) for r in rhos]
    Ns = (ctypes.c_int * max(nbox, 1))(*[int(r.shape[0]) for r in rhos])
    rp = (ctypes.c_void_p * max(nbox, 1))(*[r.data_ptr() for r in rhos])
    up = (ctypes.c_void_p * max(nbox, 1))(*[u.data_ptr() for u in us])
    pp = (mgfr_params * max(nbox, 1))(*[p.c() for p in params_list])
    for r, u in zip(rhos, us):
        assert r.is_cuda and r.is_contiguous() and u.is_cuda and u.is_contiguous()
    H = opts.max_cycles + 1
    hist = np.zeros(max(nbox, 1) * H)
    nh = np.zeros(max(nbox, 1), dtype=np.int32)
    st = lib().mg_fr_solve_batch(ctx.handle, nbox, Ns, rp, pp, ctypes.byref(opts), up,
                                 hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 nh.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _stream(stream))
    if raise_on_error and st not in (MGFR_OK, MGFR_ENOTCONV):
        raise MgfrError(st, ctx.last_error())
    hists = [hist[i * H:i * H + nh[i]].copy() for i in range(nbox)]
    return us, hists, st


TUNED_FIELDS = ("pre", "post", "inner_cycles", "planes", "tile")


def mgfr_autotune(ctx: Context, rho, params: Params, base: mgfr_opts | None = None, u_scratch=None,
                  stream=None, cache_path: str | None = None, key: str | None = None):
    """Times candidate settings (sweeps, planes per workgroup, inner cycles) on this problem and
    returns (best opts, best solve ms).  With cache_path, results are kept in a JSON file under
    `key` (default: N, precision and the GPU architecture) and reused without timing."""
    import json
    import torch
    if base is None:
        base = mgfr_default_opts()
    N = rho.shape[0]
    if key is None:
        arch = torch.cuda.get_device_properties(rho.device).gcnArchName.split(":")[0]
        key = f"N={N},precision={base.precision},arch={arch}"
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            o = mgfr_opts()
            ctypes.memmove(ctypes.byref(o), ctypes.byref(base), ctypes.sizeof(o))
            for k in TUNED_FIELDS:
                setattr(o, k, cache[key].get(k, 0))
            return o, cache[key]["ms"]
    if u_scratch is None:
        u_scratch = torch.empty_like(rho)
    best = mgfr_opts()
    ms = ctypes.c_double(0.0)
    st = lib().mgfr_autotune(ctx.handle, _ptr(rho), N, ctypes.byref(params.c()), ctypes.byref(base),
                             _ptr(u_scratch), ctypes.byref(best), ctypes.byref(ms), _stream(stream))
    if st != MGFR_OK:
        raise MgfrError(st, ctx.last_error())
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = {k: getattr(best, k) for k in TUNED_FIELDS}
        cache[key]["ms"] = ms.value
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, ms.value
