"""Python front end of the MI355X multigrid pressure-Poisson solver.

torch supplies device memory and the HIP stream; every computation runs in the
library's HIP kernels through the C ABI (include/mgp.h).  Tensors are float64,
contiguous, on the current HIP device, x fastest: cells ``[nz, ny, nx]``,
x-faces ``[nz, ny, nx+1]``, y-faces ``[nz, ny+1, nx]``, z-faces ``[nz+1, ny, nx]``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib as L
from ._lib import MgError


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor, name: str, shape: Optional[Sequence[int]] = None) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor (got {t.device})")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64 (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def face_shapes(dims: Sequence[int]) -> Tuple[Tuple[int, int, int], ...]:
    nx, ny, nz = dims
    return (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)


@dataclass
class SolveStats:
    status: int
    cycles: int
    rel_res: float
    rhs_mean_removed: float
    setup_ms: float
    solve_ms: float
    hist: List[float]
    kernel_ms: List[float] = field(default_factory=list)
    kernel_launches: List[int] = field(default_factory=list)
    kernel_bytes: List[float] = field(default_factory=list)
    kernel_ms_finest: List[float] = field(default_factory=list)
    kernel_launches_finest: List[int] = field(default_factory=list)
    kernel_bytes_finest: List[float] = field(default_factory=list)

    @classmethod
    def from_c(cls, s: L.MgStats) -> "SolveStats":
        n = min(s.cycles + 1, L.MG_HIST_MAX)
        return cls(s.status, s.cycles, s.rel_res, s.rhs_mean_removed, s.setup_ms, s.solve_ms,
                   list(s.hist[:n]), list(s.kernel_ms), list(s.kernel_launches), list(s.kernel_bytes),
                   list(s.kernel_ms_finest), list(s.kernel_launches_finest), list(s.kernel_bytes_finest))


def plan_levels(dims: Sequence[int], coarse_max: int = 4) -> int:
    return int(L.load().mg_plan_levels(L.dims_arg(dims), coarse_max))


class Solver:
    """Level hierarchy for one set of face coefficients (mg_setup).

    precision: "fp64" (FP64 V-cycles) or "mixed" (FP32 V-cycles inside an FP64
    defect-correction loop).  zero_guess: solves start from p = 0.  timing:
    record HIP-event durations of the finest-grid kernels.  level_launches: one
    launch per kernel on every level (no single-workgroup launch for the levels
    of at most 4096 cells; same results).
    """

    def __init__(self, beta_x: Optional[torch.Tensor], beta_y: Optional[torch.Tensor] = None,
                 beta_z: Optional[torch.Tensor] = None, h: float = 1.0,
                 bc: str = "neumann", precision: str = "fp64", pre: int = 2, post: int = 2,
                 max_cycles: int = 100, coarse_max: int = 4, zero_guess: bool = False,
                 timing: bool = False, stream: Optional[torch.cuda.Stream] = None, method: str = "vcycle",
                 rho: Optional[torch.Tensor] = None, level_launches: bool = False):
        self._lib = L.load()
        self._ctx = ctypes.c_void_p(None)
        if bc != "neumann":
            raise MgError(L.MG_EINVAL, f"unsupported boundary condition {bc!r}")
        if rho is not None:
            nz, ny, nx = rho.shape
            self.dims = (nx, ny, nz)
        else:
            nz, ny, nx1 = beta_x.shape
            self.dims = (nx1 - 1, ny, nz)
        self.density = rho is not None
        self.h = float(h)
        self.precision = precision
        shapes = face_shapes(self.dims)
        prec = {"fp64": L.MG_PREC_FP64, "mixed": L.MG_PREC_MIXED}.get(precision)
        if prec is None:
            raise MgError(L.MG_EINVAL, f"precision must be 'fp64' or 'mixed' (got {precision!r})")
        if method not in ("vcycle", "fcg"):
            raise MgError(L.MG_EINVAL, f"method must be 'vcycle' or 'fcg' (got {method!r})")
        self.method = method
        flags = ((L.MG_FLAG_ZERO_GUESS if zero_guess else 0) | (L.MG_FLAG_TIMING if timing else 0)
                 | (L.MG_FLAG_FCG if method == "fcg" else 0)
                 | (L.MG_FLAG_LEVEL_LAUNCHES if level_launches else 0))
        self.opts = L.MgOpts(pre, post, max_cycles, coarse_max, prec, flags)
        self._stream = stream
        self._sh = _stream_handle(stream)
        if rho is not None:
            st = self._lib.mg_setup_density(ctypes.byref(self._ctx), _ptr(rho, "rho", self.cell_shape),
                                            L.dims_arg(self.dims), self.h, L.MG_BC_NEUMANN,
                                            ctypes.byref(self.opts), self._sh)
        else:
            st = self._lib.mg_setup(ctypes.byref(self._ctx), _ptr(beta_x, "beta_x", shapes[0]),
                                    _ptr(beta_y, "beta_y", shapes[1]), _ptr(beta_z, "beta_z", shapes[2]),
                                    L.dims_arg(self.dims), self.h, L.MG_BC_NEUMANN, ctypes.byref(self.opts),
                                    self._sh)
        if st != L.MG_OK:
            self._ctx = ctypes.c_void_p(None)
            raise MgError(st, L.last_error(None))
        self.device = (rho if rho is not None else beta_x).device
        # bumped by every coefficient import (update / update_density), so that a
        # caller holding a version can tell whether the hierarchy still holds the
        # coefficients it imported
        self.coef_version = 0

    @classmethod
    def from_density(cls, rho: torch.Tensor, h: float, **kw) -> "Solver":
        """Hierarchy for the coefficients 2/(rho_L + rho_R) of a cell density
        (mg_setup_density): same results as the faces of faces_from_density(rho),
        with the finest FP64 residual passes reading rho instead of three face arrays."""
        return cls(None, None, None, h, rho=rho, **kw)

    # -- lifetime ---------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.mg_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(None)

    @property
    def closed(self) -> bool:
        return getattr(self, "_ctx", None) is None or not self._ctx.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int) -> None:
        if st != L.MG_OK:
            raise MgError(st, L.last_error(self._ctx))

    @property
    def cell_shape(self) -> Tuple[int, int, int]:
        nx, ny, nz = self.dims
        return (nz, ny, nx)

    @property
    def num_levels(self) -> int:
        n = 0
        while n < L.MG_MAX_LEVELS and self._lib.mg_level_info(self._ctx, n, None, None) == L.MG_OK:
            n += 1
        return n

    def level_info(self, level: int) -> Tuple[Tuple[int, int, int], float]:
        d = (ctypes.c_int * 3)()
        h = ctypes.c_double()
        self._check(self._lib.mg_level_info(self._ctx, level, d, ctypes.byref(h)))
        return (d[0], d[1], d[2]), h.value

    def update(self, beta_x: torch.Tensor, beta_y: torch.Tensor, beta_z: torch.Tensor) -> None:
        """New face coefficients for the same grid (no allocation)."""
        shapes = face_shapes(self.dims)
        self.coef_version += 1
        self._check(self._lib.mg_update(self._ctx, _ptr(beta_x, "beta_x", shapes[0]),
                                        _ptr(beta_y, "beta_y", shapes[1]), _ptr(beta_z, "beta_z", shapes[2])))
        self.density = False

    def update_density(self, rho: torch.Tensor) -> None:
        """New cell density (contexts made from a density only; no allocation)."""
        self.coef_version += 1
        self._check(self._lib.mg_update_density(self._ctx, _ptr(rho, "rho", self.cell_shape)))
        self.density = True

    def set_timing_classes(self, classes: Optional[Sequence[int]] = None) -> None:
        """Time only these kernel classes (MG_K_* values; None: all) in later solves
        of a context made with timing=True."""
        mask = (1 << L.MG_K_COUNT) - 1 if classes is None else sum(1 << int(k) for k in set(classes))
        self._check(self._lib.mg_set_timing_classes(self._ctx, mask))

    # -- solves -----------------------------------------------------------------
    def solve(self, rhs: torch.Tensor, tol: float = 1e-10, p: Optional[torch.Tensor] = None,
              check: bool = True) -> Tuple[torch.Tensor, SolveStats]:
        """Zero-mean p with L p = rhs - mean(rhs).  p (optional) is the initial guess, overwritten."""
        if p is None:
            p = torch.zeros(self.cell_shape, dtype=torch.float64, device=rhs.device)
        st = L.MgStats()
        status = self._lib.mg_solve(self._ctx, _ptr(rhs, "rhs", self.cell_shape), _ptr(p, "p", self.cell_shape),
                                    float(tol), ctypes.byref(st))
        stats = SolveStats.from_c(st)
        if check and status != L.MG_OK:
            raise MgError(status, L.last_error(self._ctx))
        return p, stats

    def solve_adjoint(self, g: torch.Tensor, tol: float = 1e-10, lam: Optional[torch.Tensor] = None,
                      check: bool = True) -> Tuple[torch.Tensor, SolveStats]:
        if lam is None:
            lam = torch.zeros(self.cell_shape, dtype=torch.float64, device=g.device)
        st = L.MgStats()
        status = self._lib.mg_solve_adjoint(self._ctx, _ptr(g, "g", self.cell_shape),
                                            _ptr(lam, "lambda", self.cell_shape), float(tol), ctypes.byref(st))
        stats = SolveStats.from_c(st)
        if check and status != L.MG_OK:
            raise MgError(status, L.last_error(self._ctx))
        return lam, stats

    def face_grad(self, lam: torch.Tensor, p: torch.Tensor):
        shapes = face_shapes(self.dims)
        g = [torch.empty(s, dtype=torch.float64, device=p.device) for s in shapes]
        self._check(self._lib.mg_face_grad(self._ctx, _ptr(lam, "lambda", self.cell_shape),
                                           _ptr(p, "p", self.cell_shape), *[_ptr(a, "g") for a in g]))
        return tuple(g)

    def apply(self, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty_like(x)
        self._check(self._lib.mg_apply(self._ctx, _ptr(x, "x", self.cell_shape), _ptr(y, "y")))
        return y

    # -- single kernels on one level (verification) -----------------------------
    def _level_shape(self, level: int) -> Tuple[int, int, int]:
        (nx, ny, nz), _ = self.level_info(level)
        return (nz, ny, nx)

    def level_faces(self, level: int):
        (nx, ny, nz), _ = self.level_info(level)
        g = [torch.empty(s, dtype=torch.float64, device=self.device) for s in face_shapes((nx, ny, nz))]
        self._check(self._lib.mg_level_faces(self._ctx, level, *[_ptr(a, "beta") for a in g]))
        return tuple(g)

    def smooth(self, b: torch.Tensor, p: torch.Tensor, level: int = 0, sweeps: int = 1, order: int = 0,
               precision: str = "fp64") -> torch.Tensor:
        q = p.clone()
        shp = self._level_shape(level)
        pr = L.MG_PREC_FP64 if precision == "fp64" else L.MG_PREC_MIXED
        self._check(self._lib.mg_smooth(self._ctx, level, pr, _ptr(b, "b", shp), _ptr(q, "p", shp), sweeps, order))
        return q

    def residual_restrict(self, b: torch.Tensor, p: torch.Tensor, level: int = 0,
                          precision: str = "fp64") -> torch.Tensor:
        shp = self._level_shape(level)
        out = torch.empty(self._level_shape(level + 1), dtype=torch.float64, device=b.device)
        pr = L.MG_PREC_FP64 if precision == "fp64" else L.MG_PREC_MIXED
        self._check(self._lib.mg_residual_restrict(self._ctx, level, pr, _ptr(b, "b", shp), _ptr(p, "p", shp),
                                                   _ptr(out, "b_coarse")))
        return out

    def presmooth_restrict(self, b: torch.Tensor, level: int = 0, precision: str = "fp64"):
        """The V-cycle's pre-smoothing of `level` from zero and the restriction of
        its residual: returns (p, b_coarse)."""
        shp = self._level_shape(level)
        p = torch.empty(shp, dtype=torch.float64, device=b.device)
        out = torch.empty(self._level_shape(level + 1), dtype=torch.float64, device=b.device)
        pr = L.MG_PREC_FP64 if precision == "fp64" else L.MG_PREC_MIXED
        self._check(self._lib.mg_presmooth_restrict(self._ctx, level, pr, _ptr(b, "b", shp), _ptr(p, "p", shp),
                                                    _ptr(out, "b_coarse")))
        return p, out

    def prolong_correct(self, e: torch.Tensor, p: torch.Tensor, level: int = 0,
                        precision: str = "fp64") -> torch.Tensor:
        q = p.clone()
        pr = L.MG_PREC_FP64 if precision == "fp64" else L.MG_PREC_MIXED
        self._check(self._lib.mg_prolong_correct(self._ctx, level, pr,
                                                 _ptr(e, "e", self._level_shape(level + 1)),
                                                 _ptr(q, "p", self._level_shape(level))))
        return q

    def coarse_solve(self, r: torch.Tensor) -> torch.Tensor:
        e = torch.empty_like(r)
        shp = self._level_shape(self.num_levels - 1)
        self._check(self._lib.mg_coarse_solve(self._ctx, _ptr(r, "r", shp), _ptr(e, "e", shp)))
        return e

    def residual_norm2(self, b: torch.Tensor, p: torch.Tensor) -> float:
        out = ctypes.c_double()
        self._check(self._lib.mg_residual_norm2(self._ctx, _ptr(b, "b", self.cell_shape),
                                                _ptr(p, "p", self.cell_shape), ctypes.byref(out)))
        return out.value


def solve_noalloc(beta_x: torch.Tensor, beta_y: torch.Tensor, beta_z: torch.Tensor, h: float,
                  rhs: torch.Tensor, p: torch.Tensor, tol: float = 1e-10, precision: str = "fp64",
                  pre: int = 2, post: int = 2, max_cycles: int = 100, coarse_max: int = 4,
                  zero_guess: bool = False, method: str = "vcycle", level_launches: bool = False,
                  stream: Optional[torch.cuda.Stream] = None, check: bool = True) -> SolveStats:
    """Set up and solve in one call that allocates nothing (mg_solve_noalloc): the
    hierarchy lives in the library's static per-GPU scratch buffer, so grids are
    limited to what fits in MG_NOALLOC_SCRATCH_BYTES.  p (the initial guess unless
    zero_guess) is overwritten with the solution; same results as Solver(...).solve."""
    nz, ny, nx1 = beta_x.shape
    dims = (nx1 - 1, ny, nz)
    shapes = face_shapes(dims)
    cells = (nz, ny, nx1 - 1)
    prec = {"fp64": L.MG_PREC_FP64, "mixed": L.MG_PREC_MIXED}.get(precision)
    if prec is None or method not in ("vcycle", "fcg"):
        raise MgError(L.MG_EINVAL, f"bad precision {precision!r} or method {method!r}")
    flags = ((L.MG_FLAG_ZERO_GUESS if zero_guess else 0) | (L.MG_FLAG_FCG if method == "fcg" else 0)
             | (L.MG_FLAG_LEVEL_LAUNCHES if level_launches else 0))
    opts = L.MgOpts(pre, post, max_cycles, coarse_max, prec, flags)
    st = L.MgStats()
    status = L.load().mg_solve_noalloc(_ptr(beta_x, "beta_x", shapes[0]), _ptr(beta_y, "beta_y", shapes[1]),
                                       _ptr(beta_z, "beta_z", shapes[2]), L.dims_arg(dims), float(h),
                                       L.MG_BC_NEUMANN, ctypes.byref(opts), _ptr(rhs, "rhs", cells),
                                       _ptr(p, "p", cells), float(tol), ctypes.byref(st), _stream_handle(stream))
    if check and status != L.MG_OK:
        raise MgError(status, L.last_error(None))
    return SolveStats.from_c(st)


# ---------------------------------------------------------------------------
# inputs of the solve
# ---------------------------------------------------------------------------

def faces_from_vof(f_drop: torch.Tensor, f_film: torch.Tensor, rho_drop: float, rho_film: float,
                   rho_gas: float, stream: Optional[torch.cuda.Stream] = None):
    """Face coefficients 2/(rho_L + rho_R) from the two liquid VOF fractions (GPU)."""
    nz, ny, nx = f_drop.shape
    dims = (nx, ny, nz)
    shapes = face_shapes(dims)
    out = [torch.empty(s, dtype=torch.float64, device=f_drop.device) for s in shapes]
    st = L.load().mg_faces_from_vof(_ptr(f_drop, "f_drop"), _ptr(f_film, "f_film", f_drop.shape),
                                    L.dims_arg(dims), float(rho_drop), float(rho_film), float(rho_gas),
                                    *[_ptr(a, "beta") for a in out], _stream_handle(stream))
    L.check(st)
    return tuple(out)


def density_from_vof(f_drop: torch.Tensor, f_film: torch.Tensor, rho_drop: float, rho_film: float,
                     rho_gas: float, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Cell density sum_i rho_i f_i from the two liquid VOF fractions (GPU)."""
    nz, ny, nx = f_drop.shape
    rho = torch.empty_like(f_drop)
    st = L.load().mg_density_from_vof(_ptr(f_drop, "f_drop"), _ptr(f_film, "f_film", f_drop.shape),
                                      L.dims_arg((nx, ny, nz)), float(rho_drop), float(rho_film),
                                      float(rho_gas), _ptr(rho, "rho"), _stream_handle(stream))
    L.check(st)
    return rho


def faces_from_density(rho: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
    """Face coefficients 2/(rho_L + rho_R), 0 on walls, from a cell density (GPU)."""
    nz, ny, nx = rho.shape
    shapes = face_shapes((nx, ny, nz))
    out = [torch.empty(s, dtype=torch.float64, device=rho.device) for s in shapes]
    st = L.load().mg_faces_from_density(_ptr(rho, "rho"), L.dims_arg((nx, ny, nz)),
                                        *[_ptr(a, "beta") for a in out], _stream_handle(stream))
    L.check(st)
    return tuple(out)


def density_grad(rho: torch.Tensor, g_x: torch.Tensor, g_y: torch.Tensor, g_z: torch.Tensor,
                 stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """dL/drho from dL/dbeta on the faces, through beta_f = 2/(rho_L + rho_R) (GPU)."""
    nz, ny, nx = rho.shape
    shapes = face_shapes((nx, ny, nz))
    g = torch.empty_like(rho)
    st = L.load().mg_density_grad(_ptr(rho, "rho"), L.dims_arg((nx, ny, nz)), _ptr(g_x, "g_x", shapes[0]),
                                  _ptr(g_y, "g_y", shapes[1]), _ptr(g_z, "g_z", shapes[2]), _ptr(g, "g_rho"),
                                  _stream_handle(stream))
    L.check(st)
    return g


def divergence(u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, h: float, dt: float = 1.0,
               stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """b = div_h(u, v, w)/dt on the MAC grid (GPU)."""
    nz, ny, nx1 = u.shape
    dims = (nx1 - 1, ny, nz)
    shapes = face_shapes(dims)
    b = torch.empty((nz, ny, nx1 - 1), dtype=torch.float64, device=u.device)
    st = L.load().mg_divergence(_ptr(u, "u", shapes[0]), _ptr(v, "v", shapes[1]), _ptr(w, "w", shapes[2]),
                                L.dims_arg(dims), float(h), float(dt), _ptr(b, "b"), _stream_handle(stream))
    L.check(st)
    return b


def velocity_correct(bx: torch.Tensor, by: torch.Tensor, bz: torch.Tensor, p: torch.Tensor,
                     u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, h: float, dt: float = 1.0,
                     stream: Optional[torch.cuda.Stream] = None) -> None:
    """In place on the GPU: u_f -= dt beta_f (p_R - p_L)/h on interior faces."""
    nz, ny, nx = p.shape
    dims = (nx, ny, nz)
    shapes = face_shapes(dims)
    st = L.load().mg_velocity_correct(_ptr(bx, "beta_x", shapes[0]), _ptr(by, "beta_y", shapes[1]),
                                      _ptr(bz, "beta_z", shapes[2]), _ptr(p, "p", (nz, ny, nx)),
                                      L.dims_arg(dims), float(h), float(dt), _ptr(u, "u", shapes[0]),
                                      _ptr(v, "v", shapes[1]), _ptr(w, "w", shapes[2]), _stream_handle(stream))
    L.check(st)


def vof_grad(f_drop: torch.Tensor, f_film: torch.Tensor, rho_drop: float, rho_film: float, rho_gas: float,
             g_x: torch.Tensor, g_y: torch.Tensor, g_z: torch.Tensor,
             stream: Optional[torch.cuda.Stream] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """(dL/df_drop, dL/df_film) from dL/dbeta on the faces, on the GPU."""
    nz, ny, nx = f_drop.shape
    dims = (nx, ny, nz)
    shapes = face_shapes(dims)
    gd = torch.empty_like(f_drop)
    gf = torch.empty_like(f_drop)
    st = L.load().mg_vof_grad(_ptr(f_drop, "f_drop", (nz, ny, nx)), _ptr(f_film, "f_film", (nz, ny, nx)),
                              L.dims_arg(dims), float(rho_drop), float(rho_film), float(rho_gas),
                              _ptr(g_x, "g_x", shapes[0]), _ptr(g_y, "g_y", shapes[1]), _ptr(g_z, "g_z", shapes[2]),
                              _ptr(gd, "g_drop"), _ptr(gf, "g_film"), _stream_handle(stream))
    L.check(st)
    return gd, gf
