"""MI355X-native SNAP hot path: thin ctypes binding of the libsnap C-ABI.

Every function here marshals arguments and calls the library entry point of
the same name (``include/snap.h``); all arithmetic runs in the HIP kernels.
PyTorch supplies device memory and the current HIP stream only. There is no
fallback: if the library cannot be loaded or a call fails, a ``SnapError`` is
raised.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Sequence

import numpy as np
import torch

__all__ = [
    "SnapError", "DeviceGrid", "device_grid", "lib", "workspace",
    "snap_fill_ghosts", "snap_rhs", "snap_rk3_step", "snap_cfl_dt",
    "snap_conservation_sums", "snap_conservation_sums_noalloc", "snap_workspace_bytes",
    "snap_abi_version",
    "snap_stage_timing_enable", "snap_stage_timing_read", "snap_rhs_adjoint",
    "snap_rk3_step_adjoint", "snap_rk3_step_adjoint_stages", "SNAP_OP_RHS_ADJ", "SNAP_OP_RK3_ADJ", "snap_rk3_step_cfl",
    "snap_rk3_steps_cfl", "snap_rk3_steps_status",
    "SNAP_OP_RK3_CFL",
    "snap_batched_workspace_bytes", "snap_batched_tile_variant", "snap_rk3_step_batched",
    "batched_workspace",
    "SNAP_F64", "SNAP_F32", "SNAP_BC_PERIODIC", "SNAP_BC_REFLECT",
    "SNAP_OP_RHS", "SNAP_OP_RK3", "SNAP_OP_CFL", "SNAP_OP_SUMS",
    "SNAP_EOS_PASSIVE", "SNAP_EOS_MIXTURE", "SNAP_TRACER_VAPOUR", "SNAP_TRACER_CONDENSATE",
    "SNAP_RIEMANN_LMARS", "SNAP_RIEMANN_HLLC", "SNAP_STORE_TOTAL", "SNAP_STORE_PERTURBATION",
    "snap_kessler_step", "snap_kessler_step_adjoint", "kessler_params", "snap_saturation_adjust",
    "snap_saturation_adjust_adjoint", "satadj_params",
]

PKG = os.path.dirname(os.path.abspath(__file__))
# SNAP_LIBRARY selects another build of the same C-ABI (e.g. a tuning variant)
LIB_PATH = os.environ.get("SNAP_LIBRARY") or os.path.join(PKG, "libsnap.so")

SNAP_OK = 0
SNAP_E_INVALID = -1
SNAP_E_UNSUPPORTED = -2
SNAP_E_DEVICE = -3
SNAP_E_STATE = -4
SNAP_F64 = 0
SNAP_F32 = 1
SNAP_BC_PERIODIC = 0
SNAP_BC_REFLECT = 1
SNAP_NG = 3
SNAP_MAX_TRACERS = 8
SNAP_ABI_VERSION = 13
SNAP_EOS_PASSIVE = 0
SNAP_EOS_MIXTURE = 1
SNAP_RIEMANN_LMARS = 0
SNAP_RIEMANN_HLLC = 1
SNAP_STORE_TOTAL = 0
SNAP_STORE_PERTURBATION = 1
SNAP_TRACER_VAPOUR = 0
SNAP_TRACER_CONDENSATE = 1
SNAP_OP_RHS = 0
SNAP_OP_RK3 = 1
SNAP_OP_CFL = 2
SNAP_OP_SUMS = 3
SNAP_OP_RHS_ADJ = 4
SNAP_OP_RK3_ADJ = 5
SNAP_OP_RK3_CFL = 6

_ERROR_NAMES = {
    SNAP_E_INVALID: "SNAP_E_INVALID", SNAP_E_UNSUPPORTED: "SNAP_E_UNSUPPORTED",
    SNAP_E_DEVICE: "SNAP_E_DEVICE", SNAP_E_STATE: "SNAP_E_STATE",
}


class SnapError(RuntimeError):
    """A libsnap call returned an error code."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code
        self.msg = msg


class SnapGridC(ctypes.Structure):
    """Mirror of ``snap_grid`` in include/snap.h."""
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("ng", ctypes.c_int32), ("ntracer", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3), ("weno_linear", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("gamma", ctypes.c_double), ("grav", ctypes.c_double), ("weno_eps", ctypes.c_double),
        ("rhobar_cell", ctypes.c_void_p), ("pbar_cell", ctypes.c_void_p),
        ("rhobar_face", ctypes.c_void_p), ("pbar_face", ctypes.c_void_p),
        ("eos", ctypes.c_int32), ("tracer_kind", ctypes.c_int32 * SNAP_MAX_TRACERS),
        ("tracer_eps", ctypes.c_double * SNAP_MAX_TRACERS),
        ("tracer_sigma", ctypes.c_double * SNAP_MAX_TRACERS),
        ("tracer_mu", ctypes.c_double * SNAP_MAX_TRACERS),
        ("tracer_wt", ctypes.c_double * SNAP_MAX_TRACERS), ("rd", ctypes.c_double),
        ("riemann", ctypes.c_int32), ("storage", ctypes.c_int32),
    ]


SNAP_KESSLER_MAX_SPECIES = SNAP_MAX_TRACERS // 3


class SnapKesslerSpeciesC(ctypes.Structure):
    """Mirror of ``snap_kessler_species`` in include/snap.h."""
    _fields_ = [
        ("vapour", ctypes.c_int32), ("cloud", ctypes.c_int32), ("precip", ctypes.c_int32),
        ("k1", ctypes.c_double), ("k2", ctypes.c_double), ("k3", ctypes.c_double),
        ("k4", ctypes.c_double), ("p_ref", ctypes.c_double), ("t_ref", ctypes.c_double),
        ("beta", ctypes.c_double), ("delta", ctypes.c_double),
    ]


class SnapKesslerC(ctypes.Structure):
    """Mirror of ``snap_kessler`` in include/snap.h."""
    _fields_ = [
        ("nspecies", ctypes.c_int32),
        ("species", SnapKesslerSpeciesC * SNAP_KESSLER_MAX_SPECIES),
        ("rd", ctypes.c_double), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
    ]


SNAP_SATADJ_MAX_SPECIES = SNAP_MAX_TRACERS // 2


class SnapSatAdjSpeciesC(ctypes.Structure):
    """Mirror of ``snap_satadj_species`` in include/snap.h."""
    _fields_ = [
        ("vapour", ctypes.c_int32), ("cloud", ctypes.c_int32),
        ("p_ref", ctypes.c_double), ("t_ref", ctypes.c_double),
        ("beta", ctypes.c_double), ("delta", ctypes.c_double),
    ]


class SnapSatAdjC(ctypes.Structure):
    """Mirror of ``snap_satadj`` in include/snap.h."""
    _fields_ = [
        ("nspecies", ctypes.c_int32),
        ("species", SnapSatAdjSpeciesC * SNAP_SATADJ_MAX_SPECIES),
        ("rd", ctypes.c_double), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
    ]


_P = ctypes.c_void_p
_GP = ctypes.POINTER(SnapGridC)
_SIGNATURES = {
    "snap_last_error": (ctypes.c_char_p, []),
    "snap_abi_version": (ctypes.c_int, []),
    "snap_workspace_bytes": (ctypes.c_size_t, [_GP, ctypes.c_int]),
    "snap_fill_ghosts": (ctypes.c_int, [_GP, _P, _P]),
    "snap_rhs": (ctypes.c_int, [_GP, _P, _P, _P]),
    "snap_rk3_step": (ctypes.c_int, [_GP, _P, ctypes.c_double, _P, _P]),
    "snap_rk3_step_cfl": (ctypes.c_int, [_GP, _P, ctypes.c_double, _P, _P, _P]),
    "snap_rk3_steps_cfl": (ctypes.c_int, [_GP, _P, ctypes.c_double, ctypes.c_int, _P, _P, _P]),
    "snap_rk3_steps_status": (ctypes.c_int, [_GP, _P, _P]),
    "snap_cfl_dt": (ctypes.c_int, [_GP, _P, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_double), _P]),
    "snap_conservation_sums": (ctypes.c_int, [_GP, _P, _P, ctypes.POINTER(ctypes.c_double), _P]),
    "snap_conservation_sums_noalloc": (ctypes.c_int, [_GP, _P, ctypes.POINTER(ctypes.c_double), _P]),
    "snap_rhs_adjoint": (ctypes.c_int, [_GP, _P, _P, _P, _P, _P]),
    "snap_rk3_step_adjoint": (ctypes.c_int, [_GP, _P, ctypes.c_double, _P, _P, _P]),
    "snap_rk3_step_adjoint_stages": (ctypes.c_int, [_GP, _P, _P, ctypes.c_double, _P, _P, _P]),
    "snap_batched_workspace_bytes": (ctypes.c_size_t, [_GP, ctypes.c_int]),
    "snap_batched_tile_variant": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_int),
                                                 ctypes.POINTER(ctypes.c_int)]),
    "snap_rk3_step_batched": (ctypes.c_int, [_GP, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                             ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                             ctypes.c_int, _P, _P]),
    "snap_kessler_step": (ctypes.c_int, [_GP, _P, ctypes.c_double, ctypes.POINTER(SnapKesslerC), _P]),
    "snap_kessler_step_adjoint": (ctypes.c_int, [_GP, _P, ctypes.c_double, ctypes.POINTER(SnapKesslerC),
                                                 _P, _P]),
    "snap_saturation_adjust": (ctypes.c_int, [_GP, _P, ctypes.POINTER(SnapSatAdjC), _P]),
    "snap_saturation_adjust_adjoint": (ctypes.c_int, [_GP, _P, ctypes.POINTER(SnapSatAdjC), _P, _P]),
    "snap_stage_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "snap_stage_timing_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64)]),
}

_lib = None
_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    """Load libsnap.so (building it first only if it is absent)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                from . import build as _build
                _build.build()
            handle = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGNATURES.items():
                fn = getattr(handle, name)
                fn.restype = res
                fn.argtypes = args
            version = int(handle.snap_abi_version())
            if version != SNAP_ABI_VERSION:
                raise RuntimeError(f"{LIB_PATH} has ABI version {version}, this binding needs "
                                   f"{SNAP_ABI_VERSION}: rebuild it (python -c 'import __graft_entry__ as g; g.build()')")
            _lib = handle
        return _lib


def _check(code: int):
    if code != SNAP_OK:
        raise SnapError(code, lib().snap_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class DeviceGrid:
    """A ``snap_grid`` plus device copies of its reference profiles.

    Built from plain values; ``device_grid`` builds one from any object with
    the same attribute names (nx, ny, nz, dx, dy, dz, gamma, grav, ntracer, bc,
    weno_eps, weno_linear, rhobar_cell, pbar_cell, rhobar_face, pbar_face and,
    optionally, eos, tracer_kind, tracer_eps, tracer_sigma, tracer_mu, tracer_wt, rd, riemann).
    """

    def __init__(self, nx: int, ny: int, nz: int, dx: float, dy: float, dz: float,
                 gamma: float, grav: float, ntracer: int, bc: Sequence[int],
                 weno_eps: float, weno_linear: bool, rhobar_cell, pbar_cell,
                 rhobar_face, pbar_face, dtype: torch.dtype = torch.float64,
                 device: Optional[torch.device] = None, eos: int = SNAP_EOS_PASSIVE,
                 tracer_kind: Sequence[int] = (), tracer_eps: Sequence[float] = (),
                 tracer_sigma: Sequence[float] = (), tracer_mu: Sequence[float] = (),
                 tracer_wt: Sequence[float] = (), rd: float = 0.0,
                 riemann: int = SNAP_RIEMANN_LMARS, storage: int = SNAP_STORE_TOTAL):
        if dtype not in (torch.float64, torch.float32):
            raise ValueError("dtype must be torch.float64 or torch.float32")
        device = torch.device(device or "cuda")
        self.device = device
        self.dtype = dtype
        self.nx, self.ny, self.nz, self.ntracer = int(nx), int(ny), int(nz), int(ntracer)
        refs = []
        for arr in (rhobar_cell, pbar_cell, rhobar_face, pbar_face):
            t = torch.as_tensor(np.ascontiguousarray(np.asarray(arr, dtype=np.float64)))
            refs.append(t.to(device))
        self._refs = refs
        c = SnapGridC()
        c.nx, c.ny, c.nz, c.ng = self.nx, self.ny, self.nz, SNAP_NG
        c.ntracer = self.ntracer
        c.dtype = SNAP_F64 if dtype == torch.float64 else SNAP_F32
        for d in range(3):
            c.bc[d] = int(bc[d])
        c.weno_linear = 1 if weno_linear else 0
        c.dx, c.dy, c.dz = float(dx), float(dy), float(dz)
        c.gamma, c.grav, c.weno_eps = float(gamma), float(grav), float(weno_eps)
        c.rhobar_cell, c.pbar_cell, c.rhobar_face, c.pbar_face = (r.data_ptr() for r in refs)
        c.eos = int(eos)
        for t, (k, e, sg, mu) in enumerate(zip(tracer_kind, tracer_eps, tracer_sigma, tracer_mu)):
            if t >= SNAP_MAX_TRACERS:
                raise ValueError(f"at most {SNAP_MAX_TRACERS} tracers")
            c.tracer_kind[t], c.tracer_eps[t] = int(k), float(e)
            c.tracer_sigma[t], c.tracer_mu[t] = float(sg), float(mu)
        for t, wt in enumerate(tracer_wt):
            c.tracer_wt[t] = float(wt)
        c.rd = float(rd)
        c.riemann = int(riemann)
        c.storage = int(storage)
        self.eos = int(eos)
        self.storage = int(storage)
        self.c = c

    @property
    def nvar(self) -> int:
        return 5 + self.ntracer

    @property
    def gy(self) -> int:
        return 0 if self.ny == 1 else SNAP_NG

    @property
    def shape(self):
        return (self.nvar, self.nz + 2 * SNAP_NG, self.ny + 2 * self.gy, self.nx + 2 * SNAP_NG)

    @property
    def interior_shape(self):
        return (self.nvar, self.nz, self.ny, self.nx)

    def ptr(self):
        return ctypes.byref(self.c)

    def _check_state(self, q: torch.Tensor, name: str = "q", shape=None):
        shape = tuple(shape or self.shape)
        if not isinstance(q, torch.Tensor) or q.device.type != "cuda":
            raise ValueError(f"{name} must be a CUDA (HIP) tensor")
        if q.dtype != self.dtype:
            raise ValueError(f"{name} has dtype {q.dtype}, grid expects {self.dtype}")
        if tuple(q.shape) != shape or not q.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {shape}, got {tuple(q.shape)}")


def device_grid(g, dtype: torch.dtype = torch.float64, device=None,
                storage: int = SNAP_STORE_TOTAL) -> DeviceGrid:
    """DeviceGrid of a grid description; ``storage`` picks the form of the state
    (SNAP_STORE_TOTAL or SNAP_STORE_PERTURBATION)."""
    return DeviceGrid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.gamma, g.grav, g.ntracer, g.bc,
                      g.weno_eps, g.weno_linear, g.rhobar_cell, g.pbar_cell, g.rhobar_face,
                      g.pbar_face, dtype=dtype, device=device,
                      eos=getattr(g, "eos", SNAP_EOS_PASSIVE),
                      tracer_kind=getattr(g, "tracer_kind", ()), tracer_eps=getattr(g, "tracer_eps", ()),
                      tracer_sigma=getattr(g, "tracer_sigma", ()), tracer_mu=getattr(g, "tracer_mu", ()),
                      tracer_wt=getattr(g, "tracer_wt", ()), rd=getattr(g, "rd", 0.0),
                      riemann=getattr(g, "riemann", SNAP_RIEMANN_LMARS), storage=storage)


def snap_abi_version() -> int:
    return int(lib().snap_abi_version())


def snap_workspace_bytes(grid: DeviceGrid, op: int) -> int:
    n = int(lib().snap_workspace_bytes(grid.ptr(), int(op)))
    err = lib().snap_last_error().decode()
    if n == 0 and err:
        raise SnapError(SNAP_E_INVALID, err)
    return n


def workspace(grid: DeviceGrid, op: int) -> torch.Tensor:
    """Device workspace tensor (uint8) for operation ``op``."""
    n = snap_workspace_bytes(grid, op)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=grid.device)


def snap_fill_ghosts(grid: DeviceGrid, q: torch.Tensor, stream=None) -> None:
    grid._check_state(q)
    _check(lib().snap_fill_ghosts(grid.ptr(), ctypes.c_void_p(q.data_ptr()), _stream(stream)))


def snap_rhs(grid: DeviceGrid, q: torch.Tensor, rhs: torch.Tensor, stream=None) -> None:
    grid._check_state(q)
    grid._check_state(rhs, "rhs", grid.interior_shape)
    _check(lib().snap_rhs(grid.ptr(), ctypes.c_void_p(q.data_ptr()),
                          ctypes.c_void_p(rhs.data_ptr()), _stream(stream)))


def snap_rk3_step(grid: DeviceGrid, q: torch.Tensor, dt: float, work: torch.Tensor,
                  stream=None) -> None:
    grid._check_state(q)
    if work.numel() < snap_workspace_bytes(grid, SNAP_OP_RK3):
        raise ValueError("work is smaller than snap_workspace_bytes(grid, SNAP_OP_RK3)")
    _check(lib().snap_rk3_step(grid.ptr(), ctypes.c_void_p(q.data_ptr()), ctypes.c_double(dt),
                               ctypes.c_void_p(work.data_ptr()), _stream(stream)))


def snap_rk3_step_cfl(grid: DeviceGrid, q: torch.Tensor, cfl: float, work: torch.Tensor,
                      dt_out: torch.Tensor | None = None, stream=None) -> None:
    """One SSP-RK3 step with dt = cfl / (maximum signal speed of q) formed on
    the device; dt_out (a float64 device tensor of at least one element), if
    given, receives the step's dt."""
    grid._check_state(q)
    if work.numel() < snap_workspace_bytes(grid, SNAP_OP_RK3_CFL):
        raise ValueError("work is smaller than snap_workspace_bytes(grid, SNAP_OP_RK3_CFL)")
    dptr = None
    if dt_out is not None:
        if dt_out.dtype != torch.float64 or not dt_out.is_cuda or dt_out.numel() < 1:
            raise ValueError("dt_out must be a float64 device tensor with at least one element")
        dptr = ctypes.c_void_p(dt_out.data_ptr())
    _check(lib().snap_rk3_step_cfl(grid.ptr(), ctypes.c_void_p(q.data_ptr()),
                                   ctypes.c_double(cfl), ctypes.c_void_p(work.data_ptr()),
                                   dptr, _stream(stream)))


def snap_rk3_steps_cfl(grid: DeviceGrid, q: torch.Tensor, cfl: float, nsteps: int,
                       work: torch.Tensor, dt_out: torch.Tensor | None = None,
                       stream=None) -> None:
    """nsteps SSP-RK3 steps, each with dt = cfl / (maximum signal speed of its
    state) formed on the device; dt_out (a float64 device tensor of at least
    nsteps elements), if given, receives the time steps."""
    grid._check_state(q)
    if work.numel() < snap_workspace_bytes(grid, SNAP_OP_RK3_CFL):
        raise ValueError("work is smaller than snap_workspace_bytes(grid, SNAP_OP_RK3_CFL)")
    dptr = None
    if dt_out is not None:
        if dt_out.dtype != torch.float64 or not dt_out.is_cuda or dt_out.numel() < nsteps:
            raise ValueError("dt_out must be a float64 device tensor with at least nsteps elements")
        dptr = ctypes.c_void_p(dt_out.data_ptr())
    _check(lib().snap_rk3_steps_cfl(grid.ptr(), ctypes.c_void_p(q.data_ptr()),
                                    ctypes.c_double(cfl), ctypes.c_int(nsteps),
                                    ctypes.c_void_p(work.data_ptr()), dptr, _stream(stream)))


def snap_rk3_steps_status(grid: DeviceGrid, work: torch.Tensor, stream=None) -> None:
    """Raise SnapError(SNAP_E_STATE) if a step of the last device-dt call that
    used ``work`` met a non-finite or non-positive density or pressure."""
    if work.numel() < snap_workspace_bytes(grid, SNAP_OP_RK3_CFL):
        raise ValueError("work is smaller than snap_workspace_bytes(grid, SNAP_OP_RK3_CFL)")
    _check(lib().snap_rk3_steps_status(grid.ptr(), ctypes.c_void_p(work.data_ptr()),
                                       _stream(stream)))


def snap_cfl_dt(grid: DeviceGrid, q: torch.Tensor, cfl: float, work: torch.Tensor,
                stream=None) -> float:
    grid._check_state(q)
    out = ctypes.c_double(0.0)
    _check(lib().snap_cfl_dt(grid.ptr(), ctypes.c_void_p(q.data_ptr()), ctypes.c_double(cfl),
                             ctypes.c_void_p(work.data_ptr()), ctypes.byref(out), _stream(stream)))
    return out.value


def snap_conservation_sums(grid: DeviceGrid, q: torch.Tensor, work: torch.Tensor,
                           stream=None) -> np.ndarray:
    grid._check_state(q)
    out = (ctypes.c_double * grid.nvar)()
    _check(lib().snap_conservation_sums(grid.ptr(), ctypes.c_void_p(q.data_ptr()),
                                        ctypes.c_void_p(work.data_ptr()), out, _stream(stream)))
    return np.array(out[:], dtype=np.float64)


def snap_conservation_sums_noalloc(grid: DeviceGrid, q: torch.Tensor, stream=None) -> np.ndarray:
    """snap_conservation_sums with the library's own scratch (no workspace)."""
    grid._check_state(q)
    out = (ctypes.c_double * grid.nvar)()
    _check(lib().snap_conservation_sums_noalloc(grid.ptr(), ctypes.c_void_p(q.data_ptr()), out,
                                                _stream(stream)))
    return np.array(out[:], dtype=np.float64)


def snap_rhs_adjoint(grid: DeviceGrid, q: torch.Tensor, rhs_bar: torch.Tensor,
                     q_bar: torch.Tensor, work: torch.Tensor, stream=None) -> None:
    grid._check_state(q)
    grid._check_state(rhs_bar, "rhs_bar", grid.interior_shape)
    grid._check_state(q_bar, "q_bar", grid.interior_shape)
    if work.numel() < snap_workspace_bytes(grid, SNAP_OP_RHS_ADJ):
        raise ValueError("work is smaller than snap_workspace_bytes(grid, SNAP_OP_RHS_ADJ)")
    _check(lib().snap_rhs_adjoint(grid.ptr(), ctypes.c_void_p(q.data_ptr()),
                                  ctypes.c_void_p(rhs_bar.data_ptr()),
                                  ctypes.c_void_p(q_bar.data_ptr()),
                                  ctypes.c_void_p(work.data_ptr()), _stream(stream)))


def snap_rk3_step_adjoint(grid: DeviceGrid, q_n: torch.Tensor, dt: float, q_bar: torch.Tensor,
                          work: torch.Tensor, stream=None) -> None:
    grid._check_state(q_n)
    grid._check_state(q_bar, "q_bar", grid.interior_shape)
    if work.numel() < snap_workspace_bytes(grid, SNAP_OP_RK3_ADJ):
        raise ValueError("work is smaller than snap_workspace_bytes(grid, SNAP_OP_RK3_ADJ)")
    _check(lib().snap_rk3_step_adjoint(grid.ptr(), ctypes.c_void_p(q_n.data_ptr()),
                                       ctypes.c_double(dt), ctypes.c_void_p(q_bar.data_ptr()),
                                       ctypes.c_void_p(work.data_ptr()), _stream(stream)))


def snap_rk3_step_adjoint_stages(grid: DeviceGrid, q_n: torch.Tensor, stages: torch.Tensor,
                                 dt: float, q_bar: torch.Tensor, work: torch.Tensor,
                                 stream=None) -> None:
    """Adjoint of the step whose ``snap_rk3_step`` call used ``stages`` as its workspace."""
    grid._check_state(q_n)
    grid._check_state(q_bar, "q_bar", grid.interior_shape)
    if stages.numel() < snap_workspace_bytes(grid, SNAP_OP_RK3):
        raise ValueError("stages is smaller than snap_workspace_bytes(grid, SNAP_OP_RK3)")
    if work.numel() < snap_workspace_bytes(grid, SNAP_OP_RK3_ADJ):
        raise ValueError("work is smaller than snap_workspace_bytes(grid, SNAP_OP_RK3_ADJ)")
    _check(lib().snap_rk3_step_adjoint_stages(grid.ptr(), ctypes.c_void_p(q_n.data_ptr()),
                                              ctypes.c_void_p(stages.data_ptr()),
                                              ctypes.c_double(dt),
                                              ctypes.c_void_p(q_bar.data_ptr()),
                                              ctypes.c_void_p(work.data_ptr()), _stream(stream)))


def _grid_array(grids):
    arr = (SnapGridC * len(grids))()
    for m, g in enumerate(grids):
        arr[m] = g.c
    return arr


def snap_batched_workspace_bytes(grids) -> int:
    n = int(lib().snap_batched_workspace_bytes(_grid_array(grids), len(grids)))
    if n == 0:
        raise SnapError(SNAP_E_INVALID, lib().snap_last_error().decode())
    return n


def batched_workspace(grids) -> torch.Tensor:
    return torch.empty(snap_batched_workspace_bytes(grids), dtype=torch.uint8,
                       device=grids[0].device)


def snap_batched_tile_variant(dtype: int, ntracer: int, variant: int):
    """(tx, tz) of a batched tile variant, or None if it is unavailable."""
    tx, tz = ctypes.c_int(0), ctypes.c_int(0)
    code = lib().snap_batched_tile_variant(int(dtype), int(ntracer), int(variant),
                                           ctypes.byref(tx), ctypes.byref(tz))
    if code == SNAP_E_UNSUPPORTED:
        return None
    _check(code)
    return tx.value, tz.value


def snap_rk3_step_batched(grids, qs, dts, work: torch.Tensor, variant: int = 0,
                          nblocks: int = 0, stream=None) -> None:
    if not (len(grids) == len(qs) == len(dts)) or not grids:
        raise ValueError("grids, qs and dts must be non-empty and of equal length")
    for g, q in zip(grids, qs):
        g._check_state(q)
    ptrs = (ctypes.c_void_p * len(qs))(*[q.data_ptr() for q in qs])
    dta = (ctypes.c_double * len(dts))(*[float(d) for d in dts])
    _check(lib().snap_rk3_step_batched(_grid_array(grids), len(grids), ptrs, dta, int(variant),
                                       int(nblocks), ctypes.c_void_p(work.data_ptr()),
                                       _stream(stream)))


def snap_stage_timing_enable(enable: bool) -> None:
    _check(lib().snap_stage_timing_enable(1 if enable else 0))


def snap_stage_timing_read():
    """(summed milliseconds, number of launches) of the timed stage kernels."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().snap_stage_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def kessler_params(k) -> SnapKesslerC:
    """``snap_kessler`` from any object with ``species`` (each with vapour, cloud,
    precip, k1..k4, p_ref, t_ref, beta, delta), ``rd``, ``max_iter`` and ``tol``."""
    c = SnapKesslerC()
    if len(k.species) > SNAP_KESSLER_MAX_SPECIES:
        raise ValueError(f"at most {SNAP_KESSLER_MAX_SPECIES} species")
    c.nspecies = len(k.species)
    for i, sp in enumerate(k.species):
        d = c.species[i]
        d.vapour, d.cloud, d.precip = int(sp.vapour), int(sp.cloud), int(sp.precip)
        d.k1, d.k2, d.k3, d.k4 = float(sp.k1), float(sp.k2), float(sp.k3), float(sp.k4)
        d.p_ref, d.t_ref = float(sp.p_ref), float(sp.t_ref)
        d.beta, d.delta = float(sp.beta), float(sp.delta)
    c.rd, c.max_iter, c.tol = float(k.rd), int(k.max_iter), float(k.tol)
    return c


def snap_kessler_step(grid: DeviceGrid, q: torch.Tensor, dt: float, kessler, stream=None) -> None:
    """Kessler microphysics step of length dt on the interior of q (in place)."""
    grid._check_state(q)
    params = kessler if isinstance(kessler, SnapKesslerC) else kessler_params(kessler)
    _check(lib().snap_kessler_step(grid.ptr(), ctypes.c_void_p(q.data_ptr()), ctypes.c_double(dt),
                                   ctypes.byref(params), _stream(stream)))


def snap_kessler_step_adjoint(grid: DeviceGrid, q: torch.Tensor, dt: float, kessler, q_bar: torch.Tensor,
                              stream=None) -> None:
    """q_bar <- J^T q_bar for the Kessler step of length dt from the state q (the
    state before the step; q_bar: interior layout, in place)."""
    grid._check_state(q)
    grid._check_state(q_bar, "q_bar", grid.interior_shape)
    params = kessler if isinstance(kessler, SnapKesslerC) else kessler_params(kessler)
    _check(lib().snap_kessler_step_adjoint(grid.ptr(), ctypes.c_void_p(q.data_ptr()), ctypes.c_double(dt),
                                           ctypes.byref(params), ctypes.c_void_p(q_bar.data_ptr()),
                                           _stream(stream)))


def satadj_params(adj) -> SnapSatAdjC:
    """``snap_satadj`` from any object with ``species`` (each with vapour, cloud,
    p_ref, t_ref, beta, delta), ``rd``, ``max_iter`` and ``tol``."""
    c = SnapSatAdjC()
    if len(adj.species) > SNAP_SATADJ_MAX_SPECIES:
        raise ValueError(f"at most {SNAP_SATADJ_MAX_SPECIES} species")
    c.nspecies = len(adj.species)
    for i, sp in enumerate(adj.species):
        d = c.species[i]
        d.vapour, d.cloud = int(sp.vapour), int(sp.cloud)
        d.p_ref, d.t_ref = float(sp.p_ref), float(sp.t_ref)
        d.beta, d.delta = float(sp.beta), float(sp.delta)
    c.rd, c.max_iter, c.tol = float(adj.rd), int(adj.max_iter), float(adj.tol)
    return c


def snap_saturation_adjust(grid: DeviceGrid, q: torch.Tensor, adjust, stream=None) -> None:
    """Saturation adjustment of the interior of q (in place)."""
    grid._check_state(q)
    params = adjust if isinstance(adjust, SnapSatAdjC) else satadj_params(adjust)
    _check(lib().snap_saturation_adjust(grid.ptr(), ctypes.c_void_p(q.data_ptr()),
                                        ctypes.byref(params), _stream(stream)))


def snap_saturation_adjust_adjoint(grid: DeviceGrid, q: torch.Tensor, adjust, q_bar: torch.Tensor,
                                   stream=None) -> None:
    """q_bar <- J^T q_bar for the saturation adjustment of the state q (the
    state before the adjustment; q_bar: interior layout, in place)."""
    grid._check_state(q)
    grid._check_state(q_bar, "q_bar", grid.interior_shape)
    params = adjust if isinstance(adjust, SnapSatAdjC) else satadj_params(adjust)
    _check(lib().snap_saturation_adjust_adjoint(grid.ptr(), ctypes.c_void_p(q.data_ptr()),
                                                ctypes.byref(params), ctypes.c_void_p(q_bar.data_ptr()),
                                                _stream(stream)))
