"""ctypes binding of libfind (argument marshalling only).

Every step of the solve runs in the HIP library; this module checks shapes,
dtypes and devices of torch tensors and passes their device pointers and the
current HIP stream through the C-ABI declared in include/find.h.  It raises
if the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfind.so")

FIND_OK, FIND_E_ARG, FIND_E_NOMEM, FIND_E_SINGULAR, FIND_E_DEVICE, FIND_E_UNSUPPORTED = range(6)
PREC_FP64, PREC_MIXED, PREC_MIXED_GLESS = 0, 1, 2
CPLX_4M, CPLX_3M = 0, 1
TILE_NAMES = ("32x32", "32x16", "16x32", "16x16", "wave", "2wave", "wg64x64", "8wave", "gj")
EF_FIELDS, SF_FIELDS, LF_FIELDS, ON_FIELDS, OB_FIELDS = 17, 4, 6, 2, 5
EXPORTED = ["find_plan_create", "find_plan_destroy", "find_plan_footprint", "find_plan_flops",
            "find_n_bonds", "find_solve", "find_sync_status", "find_last_error",
            "find_plan_summary", "find_plan_export", "find_plan_set_profiling", "find_plan_profile",
            "find_plan_autotune", "find_plan_get_tiles", "find_plan_set_tiles", "find_solve_scattering",
            "find_solve_scattering_bonds",
            "find_solve_noalloc"]


class FindError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libfind status {status}: {msg}")
        self.status = status


class PlanOpts(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int), ("precision", ctypes.c_int), ("max_energies", ctypes.c_int),
                ("fp64_top_levels", ctypes.c_int), ("workspace_budget", ctypes.c_size_t),
                ("complex_mode", ctypes.c_int), ("symmetric", ctypes.c_int), ("streams", ctypes.c_int),
                ("scattering", ctypes.c_int), ("half_leaves", ctypes.c_int), ("no_contacts", ctypes.c_int),
                ("reserved", ctypes.c_int * 2)]


class PlanSummary(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int) for f in
                ("Nx", "Ny", "stencil", "leaf", "n_clusters", "depth", "n_leaves", "n_elims", "n_stages",
                 "map_len", "n_leafout", "n_outbonds", "n_outnodes", "max_n", "max_s", "max_b")] + \
               [("pool_per_energy", ctypes.c_int64), ("reserved", ctypes.c_int * 8)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime; load it first so that libfind binds
        # to the same runtime instance as the tensors it is given
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1104_0623_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, st = ctypes.c_void_p, ctypes.c_int, ctypes.c_int
        L.find_plan_create.argtypes = [i32, i32, i32, ctypes.POINTER(PlanOpts), ctypes.POINTER(vp)]
        L.find_plan_create.restype = st
        L.find_plan_destroy.argtypes = [vp]; L.find_plan_destroy.restype = st
        L.find_plan_footprint.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.find_plan_footprint.restype = st
        L.find_plan_flops.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]; L.find_plan_flops.restype = st
        L.find_n_bonds.argtypes = [i32, i32, i32]; L.find_n_bonds.restype = i32
        L.find_solve.argtypes = [vp, i32] + [vp] * 9 + [vp]
        L.find_solve.restype = st
        L.find_solve_scattering.argtypes = [vp, i32] + [vp] * 11 + [vp]
        L.find_solve_scattering.restype = st
        L.find_solve_scattering_bonds.argtypes = [vp, i32] + [vp] * 13 + [vp]
        L.find_solve_scattering_bonds.restype = st
        L.find_solve_noalloc.argtypes = [vp, i32] + [vp] * 9 + [vp]
        L.find_solve_noalloc.restype = st
        L.find_sync_status.argtypes = [vp, vp]; L.find_sync_status.restype = st
        L.find_last_error.argtypes = []; L.find_last_error.restype = ctypes.c_char_p
        L.find_plan_summary.argtypes = [vp, ctypes.POINTER(PlanSummary)]; L.find_plan_summary.restype = st
        L.find_plan_export.argtypes = [vp] + [vp] * 6; L.find_plan_export.restype = st
        L.find_plan_set_profiling.argtypes = [vp, i32]; L.find_plan_set_profiling.restype = st
        L.find_plan_profile.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int)]
        L.find_plan_profile.restype = st
        L.find_plan_autotune.argtypes = [vp, i32] + [vp] * 6 + [i32, vp]; L.find_plan_autotune.restype = st
        L.find_plan_get_tiles.argtypes = [vp, vp, vp, i32, ctypes.POINTER(ctypes.c_int)]
        L.find_plan_get_tiles.restype = st
        L.find_plan_set_tiles.argtypes = [vp, vp, i32]; L.find_plan_set_tiles.restype = st
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != FIND_OK:
        raise FindError(status, lib().find_last_error().decode())


def n_bonds(Nx: int, Ny: int, stencil: int) -> int:
    return int(lib().find_n_bonds(Nx, Ny, stencil))


class Plan:
    """A FIND plan for one mesh shape (host tree + lazily created device state)."""

    def __init__(self, Nx: int, Ny: int, stencil: int = 5, leaf: int = 8, precision: int = PREC_FP64,
                 max_energies: int = 0, workspace_budget: int = 0, fp64_top_levels: int = 0,
                 complex_mode: int = CPLX_4M, symmetric: int = 0, streams: int = 0,
                 scattering: bool = False, half_leaves: bool = False, no_contacts: bool = False):
        self.Nx, self.Ny, self.stencil = Nx, Ny, stencil
        self.scattering = bool(scattering)
        self._h = ctypes.c_void_p()
        o = PlanOpts(leaf=leaf, precision=precision, max_energies=max_energies,
                     workspace_budget=workspace_budget, fp64_top_levels=fp64_top_levels,
                     complex_mode=complex_mode, symmetric=int(symmetric), streams=streams,
                     scattering=int(bool(scattering)), half_leaves=int(bool(half_leaves)),
                     no_contacts=int(bool(no_contacts)))
        _check(lib().find_plan_create(Nx, Ny, stencil, ctypes.byref(o), ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib().find_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def summary(self) -> dict:
        s = PlanSummary()
        _check(lib().find_plan_summary(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in PlanSummary._fields_ if f != "reserved"}

    def export(self) -> dict:
        s = self.summary()
        arr = lambda k: np.zeros(max(k, 1), dtype=np.int32)
        el = arr(s["n_elims"] * EF_FIELDS); mp = arr(s["map_len"] * 3); stg = arr(s["n_stages"] * SF_FIELDS)
        lo = arr(s["n_leafout"] * LF_FIELDS); on = arr(s["n_outnodes"] * ON_FIELDS); ob = arr(s["n_outbonds"] * OB_FIELDS)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().find_plan_export(self._h, p(el), p(mp), p(stg), p(lo), p(on), p(ob)))
        return dict(summary=s,
                    elims=el[: s["n_elims"] * EF_FIELDS].reshape(-1, EF_FIELDS),
                    maps=mp[: s["map_len"] * 3].reshape(-1, 3),
                    stages=stg[: s["n_stages"] * SF_FIELDS].reshape(-1, SF_FIELDS),
                    leafout=lo[: s["n_leafout"] * LF_FIELDS].reshape(-1, LF_FIELDS),
                    outnodes=on[: s["n_outnodes"] * ON_FIELDS].reshape(-1, ON_FIELDS),
                    outbonds=ob[: s["n_outbonds"] * OB_FIELDS].reshape(-1, OB_FIELDS))

    def flops_per_energy(self, want_bonds: bool = False) -> float:
        f = ctypes.c_double()
        _check(lib().find_plan_flops(self._h, int(want_bonds), ctypes.byref(f)))
        return f.value

    def set_profiling(self, enable: bool) -> None:
        _check(lib().find_plan_set_profiling(self._h, int(enable)))

    def profile(self) -> tuple[float, float, int]:
        """(elimination-kernel ms, their algorithmic flops, launches) of the most recent solve."""
        ms, fl, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(lib().find_plan_profile(self._h, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(n)))
        return ms.value, fl.value, n.value

    def tiles(self) -> list[int]:
        """Launch configuration of each stage (index into TILE_NAMES)."""
        n = ctypes.c_int()
        _check(lib().find_plan_get_tiles(self._h, None, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_int * max(1, n.value))()
        _check(lib().find_plan_get_tiles(self._h, buf, None, n.value, ctypes.byref(n)))
        return list(buf[: n.value])

    def tile_options(self) -> list[list[int]]:
        """Configurations each stage has."""
        n = ctypes.c_int()
        _check(lib().find_plan_get_tiles(self._h, None, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_int * max(1, n.value))()
        _check(lib().find_plan_get_tiles(self._h, None, buf, n.value, ctypes.byref(n)))
        return [[t for t in range(len(TILE_NAMES)) if m >> t & 1] for m in buf[: n.value]]

    def set_tiles(self, tiles) -> None:
        buf = (ctypes.c_int * max(1, len(tiles)))(*tiles)
        _check(lib().find_plan_set_tiles(self._h, buf, len(tiles)))

    def footprint(self, nE: int, want_bonds: bool = False) -> int:
        b = ctypes.c_size_t()
        _check(lib().find_plan_footprint(self._h, nE, int(want_bonds), ctypes.byref(b)))
        return b.value


def _ptr(t, name, shape, dtype):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous {dtype} of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def solve(plan: Plan, energies, H, sigma, sigma_less, diag_G, diag_Gless,
          bond_G=None, bond_Gless=None, bond_J=None, stream=None, sigma_d=None, sigma_less_d=None,
          sigma_b=None, sigma_less_b=None) -> None:
    """Enqueue one FIND solve on `stream` (default: torch's current stream).

    energies complex128 [nE]; H float64 [nst][Ny][Nx]; sigma, sigma_less complex128
    [nE][2][Nx][Nx]; diag_G, diag_Gless complex128 [nE][Ny][Nx]; optional
    bond_G, bond_Gless complex128 [nE][nbonds] and bond_J float64 [nE][nbonds].
    For a plan created with scattering=True, sigma_d and sigma_less_d complex128
    [nE][Ny][Nx] (diagonal scattering self-energies) are required, and
    sigma_b, sigma_less_b complex128 [nE][nst-1][Ny][Nx][2] (stencil-pattern
    scattering self-energies, find_solve_scattering_bonds) may be given.
    """
    if not plan.scattering and any(v is not None for v in (sigma_d, sigma_less_d, sigma_b, sigma_less_b)):
        raise ValueError("scattering self-energies given for a plan created without scattering=True")
    if (sigma_b is None) != (sigma_less_b is None):
        raise ValueError("sigma_b and sigma_less_b go together")
    import torch
    Nx, Ny = plan.Nx, plan.Ny
    nE = int(energies.shape[0])
    nst = 5 if plan.stencil == 9 else 3
    nb = n_bonds(Nx, Ny, plan.stencil)
    c128, f64 = torch.complex128, torch.float64
    args = [_ptr(energies, "energies", (nE,), c128), _ptr(H, "H", (nst, Ny, Nx), f64),
            _ptr(sigma, "sigma", (nE, 2, Nx, Nx), c128), _ptr(sigma_less, "sigma_less", (nE, 2, Nx, Nx), c128),
            _ptr(diag_G, "diag_G", (nE, Ny, Nx), c128), _ptr(diag_Gless, "diag_Gless", (nE, Ny, Nx), c128),
            _ptr(bond_G, "bond_G", (nE, nb), c128), _ptr(bond_Gless, "bond_Gless", (nE, nb), c128),
            _ptr(bond_J, "bond_J", (nE, nb), f64)]
    if stream is None:
        stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    if plan.scattering:
        if sigma_d is None or sigma_less_d is None:
            raise ValueError("a scattering plan needs sigma_d and sigma_less_d")
        d = [_ptr(sigma_d, "sigma_d", (nE, Ny, Nx), c128), _ptr(sigma_less_d, "sigma_less_d", (nE, Ny, Nx), c128)]
        if sigma_b is not None:
            bshape = (nE, nst - 1, Ny, Nx, 2)
            b = [_ptr(sigma_b, "sigma_b", bshape, c128), _ptr(sigma_less_b, "sigma_less_b", bshape, c128)]
            _check(lib().find_solve_scattering_bonds(plan.handle, nE, *args[:4], *d, *b, *args[4:], sp))
        else:
            _check(lib().find_solve_scattering(plan.handle, nE, *args[:4], *d, *args[4:], sp))
    else:
        _check(lib().find_solve(plan.handle, nE, *args, sp))


def solve_noalloc(plan: Plan, energies, H, sigma, sigma_less, diag_G, diag_Gless,
                  bond_G=None, bond_Gless=None, bond_J=None, stream=None) -> None:
    """find_solve_noalloc: as solve() for a contacts-only plan, with the
    solve's scratch in the library's fixed per-device array (no device
    allocation; the plan must have run solve() on this device before)."""
    import torch
    Nx, Ny = plan.Nx, plan.Ny
    nE = int(energies.shape[0])
    nst = 5 if plan.stencil == 9 else 3
    nb = n_bonds(Nx, Ny, plan.stencil)
    c128, f64 = torch.complex128, torch.float64
    args = [_ptr(energies, "energies", (nE,), c128), _ptr(H, "H", (nst, Ny, Nx), f64),
            _ptr(sigma, "sigma", (nE, 2, Nx, Nx), c128), _ptr(sigma_less, "sigma_less", (nE, 2, Nx, Nx), c128),
            _ptr(diag_G, "diag_G", (nE, Ny, Nx), c128), _ptr(diag_Gless, "diag_Gless", (nE, Ny, Nx), c128),
            _ptr(bond_G, "bond_G", (nE, nb), c128), _ptr(bond_Gless, "bond_Gless", (nE, nb), c128),
            _ptr(bond_J, "bond_J", (nE, nb), f64)]
    if stream is None:
        stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    _check(lib().find_solve_noalloc(plan.handle, nE, *args, sp))


def autotune(plan: Plan, energies, H, sigma, sigma_less, diag_G, diag_Gless, reps: int = 2,
             stream=None) -> list[int]:
    """Pick each stage's wave tile by timing every configuration on these
    inputs (one pass, synchronising); diag_G / diag_Gless receive that pass's
    results.  Returns the chosen configurations."""
    import torch
    Nx, Ny = plan.Nx, plan.Ny
    nE = int(energies.shape[0])
    nst = 5 if plan.stencil == 9 else 3
    c128, f64 = torch.complex128, torch.float64
    args = [_ptr(energies, "energies", (nE,), c128), _ptr(H, "H", (nst, Ny, Nx), f64),
            _ptr(sigma, "sigma", (nE, 2, Nx, Nx), c128), _ptr(sigma_less, "sigma_less", (nE, 2, Nx, Nx), c128),
            _ptr(diag_G, "diag_G", (nE, Ny, Nx), c128), _ptr(diag_Gless, "diag_Gless", (nE, Ny, Nx), c128)]
    if stream is None:
        stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    _check(lib().find_plan_autotune(plan.handle, nE, *args, int(reps), sp))
    return plan.tiles()


def sync_status(plan: Plan, stream=None) -> None:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    _check(lib().find_sync_status(plan.handle, sp))


def run_problem(plan: Plan, prob: dict, want_bonds: bool = True, device: str = "cuda") -> dict:
    """Copy a problem (numpy arrays, see paper_1104_0623_amd.inputs) to the
    device, solve, synchronise and return numpy outputs."""
    import torch
    dev = torch.device(device)
    E = torch.as_tensor(np.ascontiguousarray(prob["energies"]), device=dev)
    H = torch.as_tensor(np.ascontiguousarray(prob["H"]), device=dev)
    S = torch.as_tensor(np.ascontiguousarray(prob["sigma"]), device=dev)
    SL = torch.as_tensor(np.ascontiguousarray(prob["sigma_less"]), device=dev)
    nE, Nx, Ny = E.shape[0], plan.Nx, plan.Ny
    nb = n_bonds(Nx, Ny, plan.stencil)
    out = dict(diag_G=torch.empty((nE, Ny, Nx), dtype=torch.complex128, device=dev),
               diag_Gless=torch.empty((nE, Ny, Nx), dtype=torch.complex128, device=dev))
    if want_bonds:
        out.update(bond_G=torch.empty((nE, nb), dtype=torch.complex128, device=dev),
                   bond_Gless=torch.empty((nE, nb), dtype=torch.complex128, device=dev),
                   bond_J=torch.empty((nE, nb), dtype=torch.float64, device=dev))
    extra = {}
    for k in ("sigma_d", "sigma_less_d", "sigma_b", "sigma_less_b"):
        if k in prob:
            extra[k] = torch.as_tensor(np.ascontiguousarray(prob[k]), device=dev)
    solve(plan, E, H, S, SL, out["diag_G"], out["diag_Gless"], out.get("bond_G"), out.get("bond_Gless"),
          out.get("bond_J"), **extra)
    sync_status(plan)
    return {k: v.cpu().numpy() for k, v in out.items()}
