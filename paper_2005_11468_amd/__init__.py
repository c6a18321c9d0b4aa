"""MI355X (gfx950) batched perfectly-stirred-reactor steady-state solver.

Thin Python binding over the C ABI of libpsr.so (include/psr.h): the
functions below only marshal torch device tensors into pointers; every step
of the solve runs in the library's HIP kernels.  There is no CPU path.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (PSR_FP64, PSR_MIXED, PSR_PERSISTENT, PSR_PLAIN, STATUS_NAMES, PSRError,
                   SolveOpts, SolveStats)

__all__ = ["Mechanism", "residual", "jacobian", "lu_factor_batch", "lu_solve_batch",
           "solve_batch", "default_opts", "workspace_bytes", "autotune", "PSR_FP64", "PSR_MIXED",
           "PSR_PLAIN", "PSR_PERSISTENT", "STATUS_NAMES", "PSRError"]


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _dev_f64(t, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 device tensor")
    return t


class Mechanism:
    """A mechanism uploaded with psr_create_mechanism (host arrays copied)."""

    def __init__(self, mech: dict):
        L = _lib.load()
        f64 = lambda k: np.ascontiguousarray(mech[k], dtype=np.float64)
        i32 = lambda k: np.ascontiguousarray(mech[k], dtype=np.int32)
        self._arrays = dict(ew=f64("elem_weight"), se=i32("species_elems"), nasa=f64("nasa7"),
                            ri=i32("reac_idx"), rn=i32("reac_nu"), pi=i32("prod_idx"),
                            pn=i32("prod_nu"), A=f64("A"), beta=f64("beta"), Ea=f64("Ea"))
        a = self._arrays
        self.n_species = a["se"].shape[0]
        self.n_reactions = a["ri"].shape[0]
        dpp = lambda x: x.ctypes.data_as(_lib.dp)
        ipp = lambda x: x.ctypes.data_as(_lib.ip)
        sd = mech.get("soot")
        self._soot = None if sd is None else _lib.SootDesc(*(sd[k] for k, _ in _lib.SootDesc._fields_))
        sp = C.pointer(self._soot) if self._soot is not None else C.POINTER(_lib.SootDesc)()
        desc = _lib.MechDesc(a["se"].shape[1], self.n_species, self.n_reactions, dpp(a["ew"]),
                             ipp(a["se"]), dpp(a["nasa"]), float(mech.get("t_low", 300.0)),
                             float(mech.get("t_high", 3000.0)), ipp(a["ri"]), ipp(a["rn"]),
                             ipp(a["pi"]), ipp(a["pn"]), dpp(a["A"]), dpp(a["beta"]), dpp(a["Ea"]), sp)
        h = C.c_void_p()
        _lib.check(L.psr_create_mechanism(C.byref(desc), C.byref(h)), "psr_create_mechanism")
        self.handle = h
        self._L = L  # keeps the library reachable for __del__ at interpreter exit

    def n_unknowns(self, energy) -> int:
        return int(_lib.load().psr_num_unknowns(self.handle, _energy(energy)))

    def __del__(self):
        h, lib = getattr(self, "handle", None), getattr(self, "_L", None)
        if h is not None and lib is not None:
            lib.psr_destroy_mechanism(h)
            self.handle = None


def _check_state(mech: Mechanism, energy: bool, x, B: int, name: str = "x"):
    """x must be [n][B] with n the mechanism's unknown count (the library reads
    n rows of B values)."""
    n = mech.n_unknowns(energy)
    if tuple(x.shape) != (n, B):
        raise ValueError(f"{name} must have shape ({n}, {B}), got {tuple(x.shape)}")


def _energy(energy) -> int:
    """Energy mode of psr_conditions: False/0 isothermal, True/1 energy
    balance, 2 prescribed reactor temperature."""
    e = int(energy)
    if e not in (0, 1, 2):
        raise ValueError("energy must be 0, 1 or 2")
    return e


def _conditions(cond: dict, energy):
    P = _dev_f64(cond["P"], "P")
    tau = _dev_f64(cond["tau"], "tau")
    Tin = _dev_f64(cond["T_in"], "T_in")
    Yin = _dev_f64(cond["Y_in"], "Y_in")
    B = P.shape[0]
    if tau.shape[0] != B or Tin.shape[0] != B or Yin.shape[1] != B:
        raise ValueError("condition arrays disagree on the batch size")
    return _lib.Conditions(B, _energy(energy), _ptr(P), _ptr(tau), _ptr(Tin), _ptr(Yin))


def residual(mech: Mechanism, cond: dict, energy: bool, x, F=None, scaled=None, stream=None):
    """psr_residual: F(x) for every reactor; x, F are [n][B] float64 device tensors."""
    torch = _torch()
    c = _conditions(cond, energy)
    x = _dev_f64(x, "x")
    _check_state(mech, energy, x, c.n_reactors)
    if F is None:
        F = torch.empty_like(x)
    _check_state(mech, energy, _dev_f64(F, "F"), c.n_reactors, "F")
    st = _lib.load().psr_residual(mech.handle, C.byref(c), _ptr(x), _ptr(F),
                                  _ptr(scaled) if scaled is not None else None, _stream(stream))
    _lib.check(st, "psr_residual")
    return F


def jacobian(mech: Mechanism, cond: dict, energy: bool, x, J=None, stream=None):
    """psr_jacobian: dF/dx, [B][n][n] row-major per reactor."""
    torch = _torch()
    c = _conditions(cond, energy)
    x = _dev_f64(x, "x")
    _check_state(mech, energy, x, c.n_reactors)
    n, B = x.shape
    if J is None:
        J = torch.empty((B, n, n), dtype=torch.float64, device=x.device)
    _lib.check(_lib.load().psr_jacobian(mech.handle, C.byref(c), _ptr(x), _ptr(J), _stream(stream)),
               "psr_jacobian")
    return J


def soot_outputs(mech: Mechanism, x, out=None, stream=None):
    """psr_soot_outputs: (f_v, N [cm^-3], d [cm]) per reactor of sooting
    states x ([N + 7][B] float64 device tensor) -> [3][B]."""
    torch = _torch()
    x = _dev_f64(x, "x")
    n, B = x.shape
    if n != mech.n_species + 7:
        raise ValueError(f"x must have {mech.n_species + 7} rows (Y, T, ln M_0..ln M_5)")
    if out is None:
        out = torch.empty((3, B), dtype=torch.float64, device=x.device)
    _lib.check(_lib.load().psr_soot_outputs(mech.handle, B, _ptr(x), _ptr(out), _stream(stream)),
               "psr_soot_outputs")
    return out


def jacobian_fd(mech: Mechanism, cond: dict, energy: bool, x, J=None, work=None, stream=None):
    """psr_jacobian_fd: forward-difference dF/dx from n + 1 residual
    evaluations, [B][n][n] row-major per reactor.  work: float64 device
    scratch of at least 3 n B elements (allocated when None)."""
    torch = _torch()
    c = _conditions(cond, energy)
    x = _dev_f64(x, "x")
    _check_state(mech, energy, x, c.n_reactors)
    n, B = x.shape
    if J is None:
        J = torch.empty((B, n, n), dtype=torch.float64, device=x.device)
    if work is None:
        work = torch.empty((3 * n * B,), dtype=torch.float64, device=x.device)
    if work.dtype != torch.float64 or not work.is_contiguous() or work.numel() < 3 * n * B:
        raise ValueError("work must be a contiguous float64 tensor of at least 3 n B elements")
    _lib.check(_lib.load().psr_jacobian_fd(mech.handle, C.byref(c), _ptr(x), _ptr(J), _ptr(work),
                                           _stream(stream)), "psr_jacobian_fd")
    return J


def lu_factor_batch(A, precision=PSR_FP64, stream=None):
    """psr_lu_factor_batch on a [B][n][n] float64 tensor (in place).  Returns (A, piv, info)."""
    torch = _torch()
    A = _dev_f64(A, "A")
    B, n, _ = A.shape
    piv = torch.empty((B, n), dtype=torch.int32, device=A.device)
    info = torch.empty((B,), dtype=torch.int32, device=A.device)
    _lib.check(_lib.load().psr_lu_factor_batch(n, B, precision, _ptr(A), _ptr(piv), _ptr(info),
                                               _stream(stream)), "psr_lu_factor_batch")
    return A, piv, info


def lu_solve_batch(LU, piv, b, stream=None):
    """psr_lu_solve_batch: b ([B][n] float64) overwritten with the solutions."""
    LU = _dev_f64(LU, "LU")
    b = _dev_f64(b, "b")
    B, n, _ = LU.shape
    _lib.check(_lib.load().psr_lu_solve_batch(n, B, _ptr(LU), _ptr(piv.contiguous()), _ptr(b),
                                              _stream(stream)), "psr_lu_solve_batch")
    return b


def default_opts(**overrides) -> SolveOpts:
    o = SolveOpts()
    _lib.load().psr_default_opts(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


class _Groups:
    def __init__(self, groups):
        self.keep = []
        arr = (_lib.Group * len(groups))()
        for i, g in enumerate(groups):
            c = _conditions(g["cond"], g["energy"])
            x = _dev_f64(g["x"], "x")
            _check_state(g["mech"], g["energy"], x, c.n_reactors)
            st = g["status"]
            nl = g.get("n_lin")
            arr[i] = _lib.Group(g["mech"].handle, c, _ptr(x), _ptr(st),
                                _ptr(nl) if nl is not None else None)
            self.keep.append(g)
        self.arr = arr
        self.n = len(groups)


def workspace_bytes(groups, opts: SolveOpts) -> int:
    G = _Groups(groups)
    return int(_lib.load().psr_workspace_bytes(G.arr, G.n, C.byref(opts)))


def solve_batch(groups, opts: SolveOpts | None = None, workspace=None, stats: bool = True,
                stream=None):
    """psr_solve_batch.  groups: list of dicts with keys mech, cond (device
    tensors), energy, x ([n][B] float64, in/out), status ([B] int32), n_lin
    ([B] int32, optional).  Returns (SolveStats or None, workspace tensor)."""
    torch = _torch()
    opts = opts or default_opts()
    G = _Groups(groups)
    L = _lib.load()
    need = int(L.psr_workspace_bytes(G.arr, G.n, C.byref(opts)))
    dev = groups[0]["x"].device
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty((max(need, 1),), dtype=torch.uint8, device=dev)
    st = SolveStats() if stats else None
    r = L.psr_solve_batch(G.arr, G.n, C.byref(opts), _ptr(workspace), workspace.numel(),
                          C.byref(st) if st is not None else None, _stream(stream))
    _lib.check(r, "psr_solve_batch")
    return st, workspace


SWEEP_PARAMS = {"T_in": 0, "tau": 1}  # PSR_SWEEP_T_IN, PSR_SWEEP_TAU


def sweep_batch(group, param: str, values, opts: SolveOpts | None = None, workspace=None,
                x_path=None, status_path=None, stats: bool = True, stream=None):
    """psr_sweep_batch: a continuation sweep of one group.  param "T_in" or
    "tau"; values: [n_steps][B] float64 device tensor of that condition per
    step (group["cond"] may omit it).  group["x"] holds the initial guess and
    ends with the last step's state.  Returns (SolveStats or None, x_path
    [n_steps][n][B], status_path [n_steps][B], workspace)."""
    torch = _torch()
    if param not in SWEEP_PARAMS:
        raise ValueError(f"param must be one of {sorted(SWEEP_PARAMS)}")
    values = _dev_f64(values, "values")
    if values.dim() != 2:
        raise ValueError("values must be [n_steps][B]")
    opts = opts or default_opts()
    g = dict(group)
    cond = dict(g["cond"])
    cond.setdefault(param, values[0])
    g["cond"] = cond
    G = _Groups([g])
    B = G.arr[0].cond.n_reactors
    if values.shape[1] != B:
        raise ValueError(f"values has {values.shape[1]} reactors, the group {B}")
    steps = values.shape[0]
    n = g["mech"].n_unknowns(g["energy"])
    dev = g["x"].device
    if x_path is None:
        x_path = torch.empty((steps, n, B), dtype=torch.float64, device=dev)
    if status_path is None:
        status_path = torch.empty((steps, B), dtype=torch.int32, device=dev)
    if tuple(x_path.shape) != (steps, n, B) or x_path.dtype != torch.float64 or not x_path.is_contiguous():
        raise ValueError("x_path must be a contiguous float64 [n_steps][n][B] tensor")
    if tuple(status_path.shape) != (steps, B) or status_path.dtype != torch.int32 \
            or not status_path.is_contiguous():
        raise ValueError("status_path must be a contiguous int32 [n_steps][B] tensor")
    L = _lib.load()
    need = int(L.psr_workspace_bytes(G.arr, G.n, C.byref(opts)))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty((max(need, 1),), dtype=torch.uint8, device=dev)
    st = SolveStats() if stats else None
    r = L.psr_sweep_batch(G.arr, SWEEP_PARAMS[param], steps, _ptr(values), C.byref(opts),
                          _ptr(workspace), workspace.numel(), _ptr(x_path), _ptr(status_path),
                          C.byref(st) if st is not None else None, _stream(stream))
    _lib.check(r, "psr_sweep_batch")
    return st, x_path, status_path, workspace


def autotune(groups, opts: SolveOpts, sample: int = 4096, cache_path: str | None = None, stream=None):
    """psr_autotune: times candidate launch shapes on the first `sample`
    reactors of each group (on copies) and writes the fastest into opts
    (engine, rpw, grid_per_cu).  Returns the TuneResult."""
    G = _Groups(groups)
    res = _lib.TuneResult()
    r = _lib.load().psr_autotune(G.arr, G.n, C.byref(opts), int(sample),
                                 cache_path.encode() if cache_path else None, C.byref(res),
                                 _stream(stream))
    _lib.check(r, "psr_autotune")
    return res
