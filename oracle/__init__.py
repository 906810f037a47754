"""Plain FP64 CPU oracle for the variable-density pressure-Poisson multigrid solve.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import this module.  The GPU library never
links, loads or calls it, and the two share no code.

The arithmetic lives in ``mg_oracle.c`` (plain loops, FP64); this module only
builds it with gcc and marshals numpy arrays through ctypes.  Every function
states the passage of the paper it follows, or the reading adopted where the
paper is silent:

* cell density from phase fractions: Sec. 2, eq. "property_calculation";
* finite-volume discretisation on a Cartesian mesh: Sec. 2 (read as the
  cell-centred 7-point operator with harmonic-mean face coefficients);
* multigrid with switch levels: Sec. 4.3.2 names it without detail; the
  V-cycle components are the readings listed in ``mg_oracle.c``.

Layouts (numpy, x fastest): cells ``[nz, ny, nx]``; x-faces ``[nz, ny, nx+1]``,
y-faces ``[nz, ny+1, nx]``, z-faces ``[nz+1, ny, nx]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OR_OK, OR_EINVAL, OR_ENOMEM, OR_ENOCONV, OR_ENONFINITE = 0, -1, -2, -4, -5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off: every product rounds)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
               "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        I, D, Lg = ctypes.c_int, ctypes.c_double, ctypes.c_long
        sig = {
            "or_set_threads": (None, [I]),
            "or_get_threads": (I, []),
            "or_density": (None, [dp, dp, Lg, D, D, D, dp]),
            "or_face_coeffs": (None, [dp, I, I, I, dp, dp, dp]),
            "or_divergence": (None, [dp, dp, dp, I, I, I, D, D, dp]),
            "or_velocity_correct": (None, [dp, dp, dp, I, I, I, D, D, dp, dp, dp, dp]),
            "or_vof_grad": (I, [dp, dp, I, I, I, D, D, D, dp, dp, dp, dp, dp]),
            "or_density_grad": (None, [dp, I, I, I, dp, dp, dp, dp]),
            "or_apply": (None, [dp, dp, dp, I, I, I, D, dp, dp]),
            "or_residual": (None, [dp, dp, dp, I, I, I, D, dp, dp, dp]),
            "or_rbgs_half": (None, [dp, dp, dp, I, I, I, D, dp, dp, I]),
            "or_restrict": (None, [dp, I, I, I, dp]),
            "or_prolong_add": (None, [dp, I, I, I, dp]),
            "or_coarsen_faces": (None, [dp, dp, dp, I, I, I, dp, dp, dp]),
            "or_coarse_solve": (I, [dp, dp, dp, I, I, I, D, dp, dp]),
            "or_face_grad": (None, [dp, dp, I, I, I, D, dp, dp, dp]),
            "or_num_levels": (I, [I, I, I, I]),
            "or_solve": (I, [dp, dp, dp, I, I, I, D, dp, dp, D, I, I, I, I, dp, ip, dp, dp]),
            "or_fcg_solve": (I, [dp, dp, dp, I, I, I, D, dp, dp, D, I, I, I, I, dp, ip, dp, dp]),
            "or_vcycles": (I, [dp, dp, dp, I, I, I, D, dp, dp, I, I, I, I]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(x: np.ndarray) -> Tuple[int, int, int]:
    nz, ny, nx = x.shape
    return nx, ny, nz


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


# ---------------------------------------------------------------------------
# inputs of the solve
# ---------------------------------------------------------------------------

def density(f_drop, f_film, rho_drop, rho_film, rho_gas) -> np.ndarray:
    """rho = sum_i rho_i f_i over drop, film and (clamped) gas (Sec. 2, eq. property_calculation)."""
    fd, ff = _c(f_drop), _c(f_film)
    rho = np.empty_like(fd)
    lib().or_density(_p(fd), _p(ff), fd.size, rho_drop, rho_film, rho_gas, _p(rho))
    return rho


def face_coeffs(rho) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """beta_f = 2/(rho_L + rho_R) on interior faces (harmonic mean of 1/rho), 0 on walls."""
    rho = _c(rho)
    nx, ny, nz = _dims(rho)
    bx = np.empty((nz, ny, nx + 1))
    by = np.empty((nz, ny + 1, nx))
    bz = np.empty((nz + 1, ny, nx))
    lib().or_face_coeffs(_p(rho), nx, ny, nz, _p(bx), _p(by), _p(bz))
    return bx, by, bz


def faces_from_vof(f_drop, f_film, rho_drop, rho_film, rho_gas):
    return face_coeffs(density(f_drop, f_film, rho_drop, rho_film, rho_gas))


def divergence(u, v, w, h: float, dt: float = 1.0) -> np.ndarray:
    """b = div_h(u*)/dt on the MAC grid."""
    u, v, w = _c(u), _c(v), _c(w)
    nz, ny, nx1 = u.shape
    nx = nx1 - 1
    b = np.empty((nz, ny, nx))
    lib().or_divergence(_p(u), _p(v), _p(w), nx, ny, nz, h, dt, _p(b))
    return b


def velocity_correct(beta, p, u, v, w, h: float, dt: float = 1.0):
    """u - dt beta grad_h p on interior faces (returns corrected copies)."""
    bx, by, bz = (_c(a) for a in beta)
    p = _c(p)
    u2, v2, w2 = _c(u).copy(), _c(v).copy(), _c(w).copy()
    nx, ny, nz = _dims(p)
    lib().or_velocity_correct(_p(bx), _p(by), _p(bz), nx, ny, nz, h, dt, _p(p),
                              _p(u2), _p(v2), _p(w2))
    return u2, v2, w2


def density_grad(rho, g_beta) -> np.ndarray:
    """dL/drho from dL/dbeta (face layouts) through beta_f = 2/(rho_L + rho_R)."""
    r = _c(rho)
    gx, gy, gz = (_c(a) for a in g_beta)
    nx, ny, nz = _dims(r)
    out = np.empty_like(r)
    lib().or_density_grad(_p(r), nx, ny, nz, _p(gx), _p(gy), _p(gz), _p(out))
    return out


def vof_grad(f_drop, f_film, rho_drop: float, rho_film: float, rho_gas: float, g_beta):
    """(dL/df_drop, dL/df_film) from dL/dbeta (face layouts), by the chain rule
    through the mixture density and the harmonic-mean face coefficients."""
    fd, ff = _c(f_drop), _c(f_film)
    gx, gy, gz = (_c(a) for a in g_beta)
    nx, ny, nz = _dims(fd)
    gd, gf = np.empty_like(fd), np.empty_like(fd)
    st = lib().or_vof_grad(_p(fd), _p(ff), nx, ny, nz, rho_drop, rho_film, rho_gas,
                           _p(gx), _p(gy), _p(gz), _p(gd), _p(gf))
    if st != OR_OK:
        raise MemoryError("or_vof_grad")
    return gd, gf


# ---------------------------------------------------------------------------
# operator pieces
# ---------------------------------------------------------------------------

def apply(beta, x, h: float) -> np.ndarray:
    """y = L x with (L x)_c = sum_f beta_f (x_nb - x_c)/h^2."""
    bx, by, bz = (_c(a) for a in beta)
    x = _c(x)
    nx, ny, nz = _dims(x)
    y = np.empty_like(x)
    lib().or_apply(_p(bx), _p(by), _p(bz), nx, ny, nz, h, _p(x), _p(y))
    return y


def residual(beta, b, p, h: float) -> np.ndarray:
    bx, by, bz = (_c(a) for a in beta)
    b, p = _c(b), _c(p)
    nx, ny, nz = _dims(p)
    r = np.empty_like(p)
    lib().or_residual(_p(bx), _p(by), _p(bz), nx, ny, nz, h, _p(b), _p(p), _p(r))
    return r


def rbgs_half(beta, b, p, h: float, colour: int) -> np.ndarray:
    """One Gauss-Seidel half-sweep over colour (i+j+k) % 2 == colour; returns a new array."""
    bx, by, bz = (_c(a) for a in beta)
    b = _c(b)
    q = _c(p).copy()
    nx, ny, nz = _dims(q)
    lib().or_rbgs_half(_p(bx), _p(by), _p(bz), nx, ny, nz, h, _p(b), _p(q), int(colour))
    return q


def restrict(r) -> np.ndarray:
    r = _c(r)
    nx, ny, nz = _dims(r)
    rc = np.empty((nz // 2, ny // 2, nx // 2))
    lib().or_restrict(_p(r), nx, ny, nz, _p(rc))
    return rc


def prolong_add(e, p) -> np.ndarray:
    """p + P e (trilinear cell-centred); returns a new array."""
    e = _c(e)
    q = _c(p).copy()
    nx, ny, nz = _dims(q)
    lib().or_prolong_add(_p(e), nx, ny, nz, _p(q))
    return q


def coarsen_faces(beta):
    bx, by, bz = (_c(a) for a in beta)
    nz, ny, nx1 = bx.shape
    nx = nx1 - 1
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    cbx = np.empty((cz, cy, cx + 1))
    cby = np.empty((cz, cy + 1, cx))
    cbz = np.empty((cz + 1, cy, cx))
    lib().or_coarsen_faces(_p(bx), _p(by), _p(bz), nx, ny, nz, _p(cbx), _p(cby), _p(cbz))
    return cbx, cby, cbz


def coarse_solve(beta, r, h: float) -> np.ndarray:
    """Zero-mean e with L e = r - mean(r), from the bordered dense system."""
    bx, by, bz = (_c(a) for a in beta)
    r = _c(r)
    nx, ny, nz = _dims(r)
    e = np.empty_like(r)
    st = lib().or_coarse_solve(_p(bx), _p(by), _p(bz), nx, ny, nz, h, _p(r), _p(e))
    if st != OR_OK:
        raise RuntimeError(f"or_coarse_solve failed: {st}")
    return e


def face_grad(lam, p, h: float):
    lam, p = _c(lam), _c(p)
    nx, ny, nz = _dims(p)
    gx = np.empty((nz, ny, nx + 1))
    gy = np.empty((nz, ny + 1, nx))
    gz = np.empty((nz + 1, ny, nx))
    lib().or_face_grad(_p(lam), _p(p), nx, ny, nz, h, _p(gx), _p(gy), _p(gz))
    return gx, gy, gz


def num_levels(dims, coarse_max: int = 4) -> int:
    nx, ny, nz = dims
    return int(lib().or_num_levels(nx, ny, nz, coarse_max))


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

class OracleResult:
    def __init__(self, status, p, cycles, rel_res, hist, rhs_mean):
        self.status, self.p, self.cycles = status, p, cycles
        self.rel_res, self.hist, self.rhs_mean = rel_res, hist, rhs_mean


def solve(beta, rhs, h: float, tol: float = 1e-10, max_cycles: int = 100, pre: int = 2,
          post: int = 2, coarse_max: int = 4, p0: Optional[np.ndarray] = None,
          check: bool = True) -> OracleResult:
    """Zero-mean p with L p = rhs - mean(rhs), by V-cycles until ||r|| <= tol ||b||."""
    bx, by, bz = (_c(a) for a in beta)
    rhs = _c(rhs)
    nx, ny, nz = _dims(rhs)
    p = np.zeros_like(rhs) if p0 is None else _c(p0).copy()
    hist = np.zeros(max_cycles + 1)
    cyc = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    mu = ctypes.c_double(0.0)
    st = lib().or_solve(_p(bx), _p(by), _p(bz), nx, ny, nz, h, _p(rhs), _p(p), tol, max_cycles,
                        pre, post, coarse_max, _p(hist), ctypes.byref(cyc), ctypes.byref(rr),
                        ctypes.byref(mu))
    if check and st != OR_OK:
        raise RuntimeError(f"or_solve failed with status {st} (rr={rr.value})")
    return OracleResult(st, p, cyc.value, rr.value, hist[: cyc.value + 1].copy(), mu.value)


def fcg_solve(beta, rhs, h: float, tol: float = 1e-10, max_iters: int = 100, pre: int = 2,
              post: int = 2, coarse_max: int = 4, p0: Optional[np.ndarray] = None,
              check: bool = True) -> OracleResult:
    """Zero-mean p with L p = rhs - mean(rhs), by flexible CG preconditioned with one
    V-cycle per iteration; `cycles` of the result counts iterations."""
    bx, by, bz = (_c(a) for a in beta)
    rhs = _c(rhs)
    nx, ny, nz = _dims(rhs)
    p = np.zeros_like(rhs) if p0 is None else _c(p0).copy()
    hist = np.zeros(max_iters + 1)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    mu = ctypes.c_double(0.0)
    st = lib().or_fcg_solve(_p(bx), _p(by), _p(bz), nx, ny, nz, h, _p(rhs), _p(p), tol, max_iters,
                            pre, post, coarse_max, _p(hist), ctypes.byref(it), ctypes.byref(rr),
                            ctypes.byref(mu))
    if check and st != OR_OK:
        raise RuntimeError(f"or_fcg_solve failed with status {st} (rr={rr.value})")
    return OracleResult(st, p, it.value, rr.value, hist[: it.value + 1].copy(), mu.value)


def vcycles(beta, rhs, h: float, cycles: int, p0: Optional[np.ndarray] = None, pre: int = 2,
            post: int = 2, coarse_max: int = 4) -> np.ndarray:
    """Exactly `cycles` V-cycles from p0 (no stopping test, mean of p kept)."""
    bx, by, bz = (_c(a) for a in beta)
    rhs = _c(rhs)
    nx, ny, nz = _dims(rhs)
    p = np.zeros_like(rhs) if p0 is None else _c(p0).copy()
    st = lib().or_vcycles(_p(bx), _p(by), _p(bz), nx, ny, nz, h, _p(rhs), _p(p), cycles, pre,
                          post, coarse_max)
    if st != OR_OK:
        raise RuntimeError(f"or_vcycles failed: {st}")
    return p


def solve_adjoint(beta, g, h: float, tol: float = 1e-10, **kw) -> OracleResult:
    """lambda = zero-mean solution of L lambda = g - mean(g) (L is symmetric)."""
    return solve(beta, g, h, tol=tol, **kw)


def gradients(beta, rhs, w, h: float, tol: float = 1e-12, **kw):
    """Loss = sum(w p): returns (p, dLoss/drhs = lambda, (g_x, g_y, g_z))."""
    p = solve(beta, rhs, h, tol=tol, **kw).p
    lam = solve_adjoint(beta, w, h, tol=tol, **kw).p
    return p, lam, face_grad(lam, p, h)
