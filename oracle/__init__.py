"""TEST INFRASTRUCTURE -- the double-precision CPU oracle of the f(R) multigrid solve.

Plain, slow and independent of the GPU library: only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this package.  The
arithmetic lives in ``mgfr_oracle.c`` (compiled with gcc into ``liboracle_mgfr.so``); this
module marshals numpy arrays and chains the per-patch solves level by level, the way the
paper solves refinements after their parent level (Sec. VI.B: boundary values of a
refinement come from interpolating the coarser level's solution; the coarse solution is
kept, i.e. the coupling is one-way).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mgfr_oracle.c")
_LIB = os.environ.get("MGFR_ORACLE_LIB") or os.path.join(_HERE, "liboracle_mgfr.so")

OK, EINVAL, ENONFINITE, ENOTCONV = 0, -1, -2, -3
CUBE_PATCH_R = -1.0


def build(force: bool = True) -> str:
    """Compiles the oracle with gcc (plain -O2; OpenMP over the independent cell loops)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fopenmp", "-shared", "-fPIC", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [("omega_m", ctypes.c_double), ("omega_l", ctypes.c_double),
                ("a", ctypes.c_double), ("n", ctypes.c_double),
                ("fr0_abs", ctypes.c_double), ("box_mpc_h", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("pre", ctypes.c_int), ("post", ctypes.c_int),
                ("coarsest_n", ctypes.c_int), ("coarsest_sweeps", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("subtract_mean", ctypes.c_int),
                ("warm_start", ctypes.c_int), ("max_step", ctypes.c_double),
                ("coarsest_rtol", ctypes.c_double)]


@dataclass
class Model:
    """Hu-Sawicki f(R) model and box (Sec. II, Sec. III.A)."""
    omega_m: float = 0.24
    omega_l: float = -1.0          # negative: 1 - omega_m
    a: float = 1.0
    n: float = 1.0
    fr0_abs: float = 1e-5
    box_mpc_h: float = 64.0

    def c(self) -> _Model:
        return _Model(self.omega_m, self.omega_l, self.a, self.n, self.fr0_abs, self.box_mpc_h)


@dataclass
class Opts:
    tol: float = 1e-12
    pre: int = 2
    post: int = 2
    coarsest_n: int = 4
    coarsest_sweeps: int = 400     # cap
    max_cycles: int = 60
    subtract_mean: bool = False
    warm_start: bool = False
    max_step: float = 1.0          # 0: plain Newton step
    coarsest_rtol: float = 1e-3    # 0: always coarsest_sweeps sweeps

    def c(self) -> _Opts:
        return _Opts(self.tol, self.pre, self.post, self.coarsest_n, self.coarsest_sweeps,
                     self.max_cycles, int(self.subtract_mean), int(self.warm_start),
                     self.max_step, self.coarsest_rtol)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if "MGFR_ORACLE_LIB" not in os.environ and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_constants.argtypes = [ctypes.POINTER(_Model), ctypes.c_int, dp]
        L.orc_operator.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_double, dp,
                                   ctypes.c_double, ctypes.POINTER(_Model), dp, dp]
        L.orc_operator_at.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_double, dp,
                                      ctypes.c_double, ctypes.POINTER(_Model), ctypes.c_longlong,
                                      ctypes.POINTER(ctypes.c_longlong), dp]
        L.orc_solve.argtypes = [dp, ctypes.c_int, ctypes.POINTER(_Model), ctypes.POINTER(_Opts),
                                dp, dp, ip]
        L.orc_solve_patch.argtypes = [dp, ctypes.c_int, ctypes.c_double, dp, ctypes.POINTER(_Model),
                                      ctypes.POINTER(_Opts), dp, dp, ip]
        L.orc_patch_boundary.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, ip, ctypes.c_int, dp, dp]
        L.orc_single_grid.argtypes = [dp, ctypes.c_int, ctypes.POINTER(_Model), ctypes.c_int,
                                      ctypes.c_double, dp, ctypes.c_int, dp]
        L.orc_solve_masked.argtypes = [dp, dp, ctypes.c_int, ctypes.POINTER(_Model), ctypes.POINTER(_Opts),
                                       dp, dp, ip]
        L.orc_masked_operator.argtypes = [ctypes.c_int, dp, dp, dp, dp, ctypes.c_double,
                                          ctypes.POINTER(_Model), dp, dp]
        for f in ("orc_constants", "orc_operator", "orc_operator_at", "orc_solve", "orc_solve_patch",
                  "orc_patch_boundary", "orc_single_grid", "orc_solve_masked", "orc_masked_operator"):
            getattr(L, f).restype = ctypes.c_int
        L.orc_last_cell_updates.argtypes = []
        L.orc_last_cell_updates.restype = ctypes.c_longlong
        L.orc_threads.argtypes = []
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        # no more threads than the CPUs this process may use (a quota caps them too)
        share = cpu_share()
        if L.orc_threads() > share:
            L.orc_set_threads(share)
        _lib = L
    return _lib


def cpu_share() -> int:
    """CPUs this process may use: its affinity mask, capped by a cgroup CPU quota and by
    OMP_NUM_THREADS when set."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            quota, period = fh.read().split()[:2]
        if quota != "max":
            n = min(n, max(1, int(int(quota) // int(period))))
    except (OSError, ValueError):
        pass
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


CONST_NAMES = ("xi", "ctilde", "K", "A", "Sbar", "D", "ubar", "C")


def constants(model: Model, N: int) -> dict:
    """Derived constants of the model on an N^3 domain grid (h = 1/N)."""
    out = np.zeros(8)
    st = lib().orc_constants(ctypes.byref(model.c()), N, _dp(out))
    if st != 0:
        raise ValueError(f"orc_constants failed ({st})")
    return dict(zip(CONST_NAMES, out.tolist()))


def operator(u, model: Model, h: float, rho=None, rho_ref: float = 1.0, ub=None,
             r: float = CUBE_PATCH_R):
    """L(u) and dL/du at every cell.  rho=None: coarse-level operator (no density terms).
    ub=None: periodic grid; else ub[6,n,n] refinement boundary values, ghost mask ratio r."""
    u = _f64(u)
    n = u.shape[0]
    assert u.shape == (n, n, n)
    rho = None if rho is None else _f64(rho)
    ub = None if ub is None else _f64(ub)
    L = np.zeros_like(u)
    dL = np.zeros_like(u)
    st = lib().orc_operator(n, h, _dp(u), _dp(rho), rho_ref, _dp(ub), r, ctypes.byref(model.c()),
                            _dp(L), _dp(dL))
    if st != 0:
        raise ValueError(f"orc_operator failed ({st})")
    return L, dL


def operator_at(u, model: Model, h: float, idx, rho=None, rho_ref: float = 1.0, ub=None,
                r: float = CUBE_PATCH_R):
    """L(u) at the flat C-order cell indices idx only."""
    u = _f64(u)
    n = u.shape[0]
    rho = None if rho is None else _f64(rho)
    ub = None if ub is None else _f64(ub)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(idx.shape[0])
    st = lib().orc_operator_at(n, h, _dp(u), _dp(rho), rho_ref, _dp(ub), r, ctypes.byref(model.c()),
                               idx.shape[0], idx.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                               _dp(out))
    if st != 0:
        raise ValueError(f"orc_operator_at failed ({st})")
    return out


def restrict_mean(v):
    """8-child mean onto the level with half the cells per side."""
    v = _f64(v)
    n = v.shape[0] // 2
    return v.reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5))


def tau(u, rho, model: Model, h: float | None = None, rho_ref: float = 1.0):
    """Truncation-error estimate of Sec. V.B (the FAS relation): tau^h = L^H(R u) - R L^h(u) on
    the periodic grid, each operator with its own level's density (R rho on the coarse level)
    and cell size (H = 2h).  Written out from the definition with the oracle's operator."""
    u = _f64(u)
    n = u.shape[0]
    h = 1.0 / n if h is None else h
    LH, _ = operator(restrict_mean(u), model, 2.0 * h, rho=restrict_mean(rho), rho_ref=rho_ref)
    Lh, _ = operator(u, model, h, rho=rho, rho_ref=rho_ref)
    return LH - restrict_mean(Lh)


def solve(rho, model: Model, opts: Opts | None = None, u0=None):
    """Periodic domain-grid solve.  Returns (u, residual history, status)."""
    opts = opts or Opts()
    rho = _f64(rho)
    N = rho.shape[0]
    u = np.zeros_like(rho) if u0 is None else _f64(u0).copy()
    if u0 is not None:
        opts = Opts(**{**opts.__dict__, "warm_start": True})
    hist = np.zeros(opts.max_cycles + 1)
    nh = ctypes.c_int(0)
    st = lib().orc_solve(_dp(rho), N, ctypes.byref(model.c()), ctypes.byref(opts.c()), _dp(u),
                         _dp(hist), ctypes.byref(nh))
    return u, hist[:nh.value].copy(), st


def solve_patch(rho, h: float, ub, model: Model, u0, opts: Opts | None = None):
    """One cube patch with fixed boundary values ub[6,n,n], started from u0."""
    opts = opts or Opts()
    rho = _f64(rho)
    n = rho.shape[0]
    u = _f64(u0).copy()
    ub = _f64(ub)
    hist = np.zeros(opts.max_cycles + 1)
    nh = ctypes.c_int(0)
    st = lib().orc_solve_patch(_dp(rho), n, h, _dp(ub), ctypes.byref(model.c()),
                               ctypes.byref(opts.c()), _dp(u), _dp(hist), ctypes.byref(nh))
    return u, hist[:nh.value].copy(), st


def patch_boundary(parent_u, porigin, parent_periodic: bool, origin, n: int):
    """(ub[6,n,n], u0[n,n,n]) of a patch from the parent level's solution."""
    pu = _f64(parent_u)
    pn = pu.shape[0]
    po = (ctypes.c_int * 3)(*[int(x) for x in porigin])
    co = (ctypes.c_int * 3)(*[int(x) for x in origin])
    ub = np.zeros((6, n, n))
    u0 = np.zeros((n, n, n))
    st = lib().orc_patch_boundary(_dp(pu), pn, po, int(parent_periodic), co, n, _dp(ub), _dp(u0))
    if st != 0:
        raise ValueError(f"orc_patch_boundary failed ({st})")
    return ub, u0


def solve_patches(u_domain, patches, rho_patches, model: Model, opts: Opts | None = None):
    """All refinement patches, level by level after their parent (Sec. VI.B).

    patches: list of dicts {level, parent, origin (level cells), n}; parent = -1 means the
    periodic domain grid (level 0), otherwise an index into patches with level - 1.
    rho_patches: list of n^3 arrays.  Returns (list of u, list of histories, list of status).
    """
    opts = opts or Opts()
    N0 = np.asarray(u_domain).shape[0]
    global last_patch_updates
    last_patch_updates = 0
    order = sorted(range(len(patches)), key=lambda p: patches[p]["level"])
    us = [None] * len(patches)
    hs = [None] * len(patches)
    sts = [None] * len(patches)
    for p in order:
        P = patches[p]
        lev, n = P["level"], P["n"]
        h = 1.0 / (N0 * 2 ** lev)
        if P["parent"] < 0:
            pu, po, per = u_domain, (0, 0, 0), True
        else:
            Q = patches[P["parent"]]
            pu, po, per = us[P["parent"]], Q["origin"], False
        ub, u0 = patch_boundary(pu, po, per, P["origin"], n)
        us[p], hs[p], sts[p] = solve_patch(rho_patches[p], h, ub, model, u0, opts)
        last_patch_updates += last_cell_updates()
    return us, hs, sts


# smoother cell visits of the last solve_patches call, all patches (timing reports only)
last_patch_updates = 0


def threads() -> int:
    """Host threads the oracle's loops use (results do not depend on it)."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Sets the oracle's host thread count (n > 0)."""
    lib().orc_set_threads(int(n))


def last_cell_updates() -> int:
    """Smoother cell visits of the last oracle solve (timing reports only)."""
    return int(lib().orc_last_cell_updates())


def single_grid(rho, model: Model, u0, nsweeps: int, subtract_mean: bool = False,
                max_step: float = 0.0):
    """Single-grid red-black Newton-Gauss-Seidel; returns (u, rms residual after each sweep)."""
    rho = _f64(rho)
    u = _f64(u0).copy()
    hist = np.zeros(nsweeps + 1)
    st = lib().orc_single_grid(_dp(rho), rho.shape[0], ctypes.byref(model.c()), int(subtract_mean),
                               max_step, _dp(u), nsweeps, _dp(hist))
    if st != 0:
        raise ValueError(f"orc_single_grid failed ({st})")
    return u, hist


def solve_masked(rho, mask, model: Model, u0, opts: Opts | None = None):
    """A refinement level with the mask scheme (Sec. V): periodic N^3 grid of the level's
    resolution, mask in [-1, 1] (active where > 0), u0 = initial guess in active cells and the
    fixed values from the coarser level elsewhere.  Returns (u, residual history, status)."""
    opts = opts or Opts()
    rho = _f64(rho)
    mask = _f64(mask)
    u = _f64(u0).copy()
    N = rho.shape[0]
    hist = np.zeros(opts.max_cycles + 1)
    nh = ctypes.c_int(0)
    st = lib().orc_solve_masked(_dp(rho), _dp(mask), N, ctypes.byref(model.c()), ctypes.byref(opts.c()),
                                _dp(u), _dp(hist), ctypes.byref(nh))
    return u, hist[:nh.value].copy(), st


def masked_operator(u, w, mask, model: Model, rho=None, rho_ref: float = 1.0):
    """(L, dL/du) of the masked operator at active cells (zero elsewhere), fixed values w."""
    u, w, mask = _f64(u), _f64(w), _f64(mask)
    rho = None if rho is None else _f64(rho)
    n = u.shape[0]
    L = np.zeros_like(u)
    dL = np.zeros_like(u)
    st = lib().orc_masked_operator(n, _dp(u), _dp(w), _dp(mask), _dp(rho), rho_ref, ctypes.byref(model.c()),
                                   _dp(L), _dp(dL))
    if st != 0:
        raise ValueError(f"orc_masked_operator failed ({st})")
    return L, dL
