"""Python face of the chanflow C ABI: argument checks and pointer marshalling
for torch tensors on the GPU.  All arithmetic runs in libchanflow.so."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


class Plan:
    """Plan for one grid: nx x ny x nz cells, periodic lengths lx, lz, wall-normal
    faces y_faces (ny+1 values).  precision: 'fp64' or 'mixed'.  y_solver:
    'pdd' (partitioned tridiagonal solve) or 'dct' (transform along y; uniform
    faces and FP64 only).  n_parts / lines_per_block: partitions per line and
    lines per block of the partitioned solve (0: automatic); tune_parts: choose
    both by timing every admissible pair at creation (see partition_timings).
    drop_parts: outer partitions G of the dropped reduced system (groups of
    n_parts/G partitions, exact inside; 0: automatic).  drop_tol < 0: default."""

    def __init__(self, nx: int, ny: int, nz: int, lx: float, lz: float, y_faces,
                 precision: str = "fp64", n_parts: int = 0, drop_tol: float = -1.0,
                 fp64_kx: int = 4, fp64_kz: int = 4, refine_passes: int = 1,
                 step: bool = False, adjoint: bool = False, y_solver: str = "pdd",
                 lines_per_block: int = 0, tune_parts: bool = False, drop_parts: int = 0, device=None):
        lib = L.lib()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.nkx = self.nx // 2 + 1
        self.lx, self.lz = float(lx), float(lz)
        yf = np.ascontiguousarray(np.asarray(y_faces, dtype=np.float64))
        if yf.shape != (self.ny + 1,):
            raise ValueError(f"y_faces must have ny+1 = {self.ny + 1} values, got {yf.shape}")
        self.y_faces = yf
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        self.precision = precision
        opt = L.cf_options()
        lib.cf_options_default(C.byref(opt))
        opt.precision = L.CF_FP64 if precision == "fp64" else L.CF_MIXED
        opt.n_parts = int(n_parts)
        opt.drop_tol = float(drop_tol)
        opt.fp64_kx = int(fp64_kx)
        opt.fp64_kz = int(fp64_kz)
        opt.refine_passes = int(refine_passes)
        opt.lines_per_block = int(lines_per_block)
        opt.drop_parts = int(drop_parts)
        if y_solver not in ("pdd", "dct"):
            raise ValueError("y_solver must be 'pdd' or 'dct'")
        opt.flags = (L.CF_PLAN_STEP if (step or adjoint) else 0) | (L.CF_PLAN_ADJOINT if adjoint else 0) \
            | (L.CF_PLAN_Y_DCT if y_solver == "dct" else 0) | (L.CF_PLAN_TUNE_PARTS if tune_parts else 0)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.cf_plan_create(C.byref(self._h), self.nx, self.ny, self.nz, self.lx, self.lz,
                                    yf.ctypes.data_as(C.POINTER(C.c_double)), C.byref(opt))
        L.check(st, "cf_plan_create")
        self.spec_dtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.state_dtype = torch.float64 if precision == "fp64" else torch.float32

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().cf_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ info
    def info(self) -> dict:
        inf = L.cf_plan_info()
        L.check(L.lib().cf_plan_query(self._h, C.byref(inf)), "cf_plan_query")
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def partition_timings(self) -> list:
        """[(n_parts, lines_per_block, mean us per launch)] timed at creation by a
        tune_parts plan, in the order timed; [] otherwise."""
        n = C.c_int()
        L.check(L.lib().cf_plan_tuning(self._h, 0, C.byref(n), None, None, None), "cf_plan_tuning")
        cnt = n.value
        if cnt == 0:
            return []
        parts, lbs, us = (C.c_int * cnt)(), (C.c_int * cnt)(), (C.c_double * cnt)()
        L.check(L.lib().cf_plan_tuning(self._h, cnt, C.byref(n), parts, lbs, us), "cf_plan_tuning")
        return [(parts[q], lbs[q], us[q]) for q in range(cnt)]

    # ------------------------------------------------------------------ timing
    def numeric_status(self) -> bool:
        """Waits for the current stream; True when no pressure solve since the
        last call saw a non-finite right-hand side (the check is cleared)."""
        st = L.lib().cf_plan_numeric_status(self._h, _stream())
        if st == L.CF_ERR_NUMERIC:
            return False
        L.check(st, "cf_plan_numeric_status")
        return True

    def set_timing(self, enable: bool):
        L.check(L.lib().cf_plan_set_timing(self._h, int(bool(enable))), "cf_plan_set_timing")

    def reset_timing(self):
        L.check(L.lib().cf_plan_reset_timing(self._h), "cf_plan_reset_timing")

    def timings(self) -> dict:
        """{kernel name: (total ms, launches)} since the last reset."""
        out = {}
        for k, name in enumerate(L.KERNELS):
            ms, n = C.c_double(), C.c_longlong()
            L.check(L.lib().cf_plan_get_timing(self._h, k, C.byref(ms), C.byref(n)), "cf_plan_get_timing")
            out[name] = (ms.value, n.value)
        return out

    # ------------------------------------------------------------------ checks
    @property
    def shape(self):
        return (self.ny, self.nz, self.nx)

    @property
    def spec_shape(self):
        return (self.nkx, self.ny, self.nz)

    def _field(self, t: torch.Tensor, name: str, dtype=torch.float64):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}, got {t.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != self.shape:
            raise ValueError(f"{name} must have shape {self.shape}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _spec(self, t: torch.Tensor, name: str):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device != self.device or t.dtype != self.spec_dtype:
            raise TypeError(f"{name} must be {self.spec_dtype} on {self.device}")
        if tuple(t.shape) != self.spec_shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.spec_shape}")
        return t

    def _new(self, dtype=torch.float64):
        return torch.empty(self.shape, dtype=dtype, device=self.device)

    # ------------------------------------------------------------------ calls
    def poisson_solve(self, f: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._field(f, "f")
        out = self._new() if out is None else self._field(out, "out")
        L.check(L.lib().cf_poisson_solve(self._h, _ptr(f), _ptr(out), _stream()), "cf_poisson_solve")
        return out

    def divergence(self, u, v, w, scale: float = 1.0, out=None) -> torch.Tensor:
        for t, n in ((u, "u"), (v, "v"), (w, "w")):
            self._field(t, n)
        out = self._new() if out is None else self._field(out, "out")
        L.check(L.lib().cf_divergence(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(out), float(scale),
                                      _stream()), "cf_divergence")
        return out

    def projection_step(self, u, v, w, dt: float, nu: float, fx: float, out=None, p=None):
        """One RK2 + pressure-projection step; returns (u1, v1, w1).  out: optional
        (u1, v1, w1) tensors (may be u, v, w themselves); p: optional float64
        tensor receiving the pressure."""
        sd = self.state_dtype
        for t, n in ((u, "u"), (v, "v"), (w, "w")):
            self._field(t, n, sd)
        if out is None:
            out = (self._new(sd), self._new(sd), self._new(sd))
        for t, n in zip(out, ("u1", "v1", "w1")):
            self._field(t, n, sd)
        pp = None if p is None else _ptr(self._field(p, "p"))
        L.check(L.lib().cf_projection_step(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(out[0]), _ptr(out[1]),
                                           _ptr(out[2]), pp, float(dt), float(nu), float(fx), _stream()),
                "cf_projection_step")
        return out

    def rk2_predictor(self, u, v, w, dt: float, nu: float, fx: float, out=None):
        """The RK2 predictor u* of a projection step alone (test hook); returns
        (us, vs, ws).  out may be (u, v, w) themselves."""
        sd = self.state_dtype
        for t, n in ((u, "u"), (v, "v"), (w, "w")):
            self._field(t, n, sd)
        if out is None:
            out = (self._new(sd), self._new(sd), self._new(sd))
        for t, n in zip(out, ("us", "vs", "ws")):
            self._field(t, n, sd)
        L.check(L.lib().cf_rk2_predictor(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(out[0]), _ptr(out[1]),
                                         _ptr(out[2]), float(dt), float(nu), float(fx), _stream()),
                "cf_rk2_predictor")
        return out

    def plane_stats(self, u, v, w, out=None):
        """Per-plane means of u, v, w and of their squares: a float64 (ny, 6)
        tensor [<u>, <v>, <w>, <u^2>, <v^2>, <w^2>]."""
        sd = self.state_dtype
        for t, n in ((u, "u"), (v, "v"), (w, "w")):
            self._field(t, n, sd)
        if out is None:
            out = torch.empty(self.ny, 6, dtype=torch.float64, device=self.device)
        if out.shape != (self.ny, 6) or out.dtype != torch.float64 or not out.is_contiguous() or out.device != self.device:
            raise ValueError("stats must be a contiguous float64 (ny, 6) tensor on the plan's device")
        L.check(L.lib().cf_plane_stats(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(out), _stream()), "cf_plane_stats")
        return out

    def run_steps(self, u, v, w, nsteps: int, dt: float, nu: float, fx: float, work=None,
                  stats_every: int = 0, stats=None, p=None, use_graph: bool = False):
        """A time loop of nsteps projection steps.  The state alternates between
        (u, v, w) and `work` (three more arrays; allocated when None); returns the
        newest state (u, v, w) or work, which holds it.  stats: float64 (ny, 6)
        accumulator that gains the plane statistics after every stats_every-th
        step.  use_graph: replay the steps from HIP graphs."""
        sd = self.state_dtype
        for t, n in ((u, "u"), (v, "v"), (w, "w")):
            self._field(t, n, sd)
        if work is None:
            work = (self._new(sd), self._new(sd), self._new(sd))
        for t, n in zip(work, ("u2", "v2", "w2")):
            self._field(t, n, sd)
        sp = None
        if stats_every > 0:
            if stats is None or stats.shape != (self.ny, 6) or stats.dtype != torch.float64 \
                    or not stats.is_contiguous() or stats.device != self.device:
                raise ValueError("stats must be a contiguous float64 (ny, 6) tensor on the plan's device")
            sp = _ptr(stats)
        pp = None if p is None else _ptr(self._field(p, "p"))
        L.check(L.lib().cf_run_steps(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(work[0]), _ptr(work[1]),
                                     _ptr(work[2]), int(nsteps), float(dt), float(nu), float(fx), int(stats_every),
                                     sp, pp, int(bool(use_graph)), _stream()), "cf_run_steps")
        return (u, v, w) if nsteps % 2 == 0 else tuple(work)

    def projection_step_adjoint(self, u, v, w, gu1, gv1, gw1, dt: float, nu: float, fx: float, out=None):
        """dJ/d(u, v, w) of one projection step from dJ/d(u1, v1, w1)."""
        sd = self.state_dtype
        for t, n in ((u, "u"), (v, "v"), (w, "w"), (gu1, "gu1"), (gv1, "gv1"), (gw1, "gw1")):
            self._field(t, n, sd)
        if out is None:
            out = (self._new(sd), self._new(sd), self._new(sd))
        for t, n in zip(out, ("gu", "gv", "gw")):
            self._field(t, n, sd)
        L.check(L.lib().cf_projection_step_adjoint(
            self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(gu1), _ptr(gv1), _ptr(gw1), _ptr(out[0]), _ptr(out[1]),
            _ptr(out[2]), float(dt), float(nu), float(fx), _stream()), "cf_projection_step_adjoint")
        return out

    def rhs_adjoint(self, u, v, w, lu, lv, lw, nu: float):
        """J_R(u, v, w)^T (lu, lv, lw) (test hook)."""
        sd = self.state_dtype
        for t, n in ((u, "u"), (v, "v"), (w, "w"), (lu, "lu"), (lv, "lv"), (lw, "lw")):
            self._field(t, n, sd)
        out = (self._new(sd), self._new(sd), self._new(sd))
        L.check(L.lib().cf_rhs_adjoint(self._h, _ptr(u), _ptr(v), _ptr(w), _ptr(lu), _ptr(lv), _ptr(lw),
                                       _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), float(nu), _stream()),
                "cf_rhs_adjoint")
        return out

    def forward_spectral(self, f: torch.Tensor, out=None) -> torch.Tensor:
        self._field(f, "f")
        out = torch.empty(self.spec_shape, dtype=self.spec_dtype, device=self.device) if out is None \
            else self._spec(out, "out")
        L.check(L.lib().cf_forward_spectral(self._h, _ptr(f), _ptr(out), _stream()), "cf_forward_spectral")
        return out

    def inverse_spectral(self, fhat: torch.Tensor, out=None) -> torch.Tensor:
        """Inverse transforms of a spectrum of shape (nx/2+1, ny, nz)."""
        self._spec(fhat, "fhat")
        out = self._new() if out is None else self._field(out, "out")
        L.check(L.lib().cf_inverse_spectral(self._h, _ptr(fhat), _ptr(out), _stream()), "cf_inverse_spectral")
        return out

    def solve_spectral(self, fhat: torch.Tensor, out=None) -> torch.Tensor:
        self._spec(fhat, "fhat")
        out = torch.empty_like(fhat) if out is None else self._spec(out, "out")
        L.check(L.lib().cf_solve_spectral(self._h, _ptr(fhat), _ptr(out), _stream()), "cf_solve_spectral")
        return out

    def solve_spectral_slabs(self, fhat: torch.Tensor, n_slabs: int, out=None, iface=None) -> torch.Tensor:
        """solve_spectral split into n_slabs y-slabs (local passes, interface
        buffer, finishing passes), as the solve would run across n_slabs
        devices.  iface: uint8 device buffer of info()['slab_iface_bytes']
        (allocated when None)."""
        self._spec(fhat, "fhat")
        out = torch.empty_like(fhat) if out is None else self._spec(out, "out")
        need = self.info()["slab_iface_bytes"]
        if iface is None:
            iface = torch.empty(need, dtype=torch.uint8, device=self.device)
        elif iface.device != self.device or iface.numel() * iface.element_size() < need or not iface.is_contiguous():
            raise ValueError(f"iface must be a contiguous device buffer of at least {need} bytes")
        L.check(L.lib().cf_solve_spectral_slabs(self._h, int(n_slabs), _ptr(fhat), _ptr(out), _ptr(iface),
                                                _stream()), "cf_solve_spectral_slabs")
        return out

    def solve_spectral_slabs_noalloc(self, fhat: torch.Tensor, n_slabs: int, out: torch.Tensor) -> torch.Tensor:
        """solve_spectral_slabs with the interface rows in the library's static
        device array (no device allocation in the call; out must be given)."""
        self._spec(fhat, "fhat")
        self._spec(out, "out")
        L.check(L.lib().cf_solve_spectral_slabs_noalloc(self._h, int(n_slabs), _ptr(fhat), _ptr(out), _stream()),
                "cf_solve_spectral_slabs_noalloc")
        return out
