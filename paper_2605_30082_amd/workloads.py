"""Seeded synthetic inputs for the variable-density pressure-Poisson solve.

This module produces raw inputs only:

* VOF volume fractions of a drop phase and a film phase, obtained by
  sampling each cell at 4x4x4 sub-cell centres against analytic shapes
  (spheres, an oblate spheroid, a flat film);
* a random face-centred intermediate velocity u* (MAC layout) with zero
  normal velocity on the domain boundary;
* loss weights for the differentiable solve.

It holds none of the solver's arithmetic: densities, face coefficients and
the discrete divergence are computed from these inputs by the solver library
and, independently, by the CPU oracle.  The phase densities below are the
values of the workloads (water drop, silicone-oil S50 film, air); the paper's
material table lists water 1000, S50 960 and air 1.225 kg/m^3, the workloads
use 1.2 for air.

Layouts: cell arrays are numpy ``[nz, ny, nx]`` (x fastest); the velocity
components are ``u [nz, ny, nx+1]``, ``v [nz, ny+1, nx]``, ``w [nz+1, ny, nx]``
where index ``i`` of ``u`` is the x-face between cells ``i-1`` and ``i``.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

RHO_DROP = 1000.0   # water
RHO_FILM = 960.0    # silicone oil S50
RHO_GAS = 1.2       # air, as the workloads specify

SEED_VELOCITY = 0
SEED_DROPS = 1
SEED_WEIGHTS = 2
SEED_FD = 3

SUB = 4  # sub-samples per cell and axis


def _sub_offsets() -> np.ndarray:
    # sub-cell centres (a + 1/2)/4, a = 0..3: dyadic, exact in binary floating point
    return (np.arange(SUB, dtype=np.float64) + 0.5) / SUB


def _axis_samples(lo: int, hi: int, n: int) -> np.ndarray:
    """Sample coordinates for cells lo..hi-1 of an axis with n cells, shape [hi-lo, 4]."""
    h = 1.0 / n
    cells = np.arange(lo, hi, dtype=np.float64)[:, None]
    return (cells + _sub_offsets()[None, :]) * h


def _fraction_in_box(n: Tuple[int, int, int], box: Tuple[Tuple[int, int], ...],
                     inside: Callable[[np.ndarray, np.ndarray, np.ndarray], np.ndarray]
                     ) -> np.ndarray:
    """Fraction of the 64 sub-samples with inside(x,y,z) true, for cells in box.

    box = ((k0,k1),(j0,j1),(i0,i1)); returns an array [k1-k0, j1-j0, i1-i0].
    """
    nx, ny, nz = n
    (k0, k1), (j0, j1), (i0, i1) = box
    zs = _axis_samples(k0, k1, nz)   # [K,4]
    ys = _axis_samples(j0, j1, ny)   # [J,4]
    xs = _axis_samples(i0, i1, nx)   # [I,4]
    out = np.zeros((k1 - k0, j1 - j0, i1 - i0), dtype=np.float64)
    # loop over the 64 sub-sample offsets, vectorised over cells
    for c in range(SUB):
        z = zs[:, c][:, None, None]
        for b in range(SUB):
            y = ys[:, b][None, :, None]
            for a in range(SUB):
                x = xs[:, a][None, None, :]
                out += inside(x, y, z)
    return out / float(SUB ** 3)


def _bbox(n: int, lo: float, hi: float) -> Tuple[int, int]:
    """Cell range [a,b) of an axis with n cells that can hold samples in (lo, hi)."""
    a = max(0, int(np.floor(lo * n)) - 1)
    b = min(n, int(np.ceil(hi * n)) + 1)
    return a, b


def ellipsoid_fraction(dims: Sequence[int], centre: Sequence[float],
                       semi_axes: Sequence[float], out: Optional[np.ndarray] = None
                       ) -> np.ndarray:
    """Add the sampled volume fraction of an axis-aligned ellipsoid to ``out``.

    A sub-sample is inside when sum(((x_d - c_d)/a_d)^2) < 1 (strict).
    Only cells in the ellipsoid's bounding box are sampled.
    """
    nx, ny, nz = dims
    if out is None:
        out = np.zeros((nz, ny, nx), dtype=np.float64)
    cx, cy, cz = centre
    ax, ay, az = semi_axes
    box = (_bbox(nz, cz - az, cz + az), _bbox(ny, cy - ay, cy + ay), _bbox(nx, cx - ax, cx + ax))
    if min(b - a for a, b in box) <= 0:
        return out

    if ax == ay == az:
        r2 = ax * ax

        def inside(x, y, z):
            return ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) < r2
    else:
        def inside(x, y, z):
            return (((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2 + ((z - cz) / az) ** 2) < 1.0

    frac = _fraction_in_box((nx, ny, nz), box, inside)
    (k0, k1), (j0, j1), (i0, i1) = box
    out[k0:k1, j0:j1, i0:i1] += frac
    return out


def sphere_fraction(dims, centre, radius, out=None):
    return ellipsoid_fraction(dims, centre, (radius, radius, radius), out)


def film_fraction(dims: Sequence[int], height: float) -> np.ndarray:
    """Sampled fraction of the layer z < height (strict); constant per z-layer."""
    nx, ny, nz = dims
    zs = _axis_samples(0, nz, nz)                      # [nz, 4]
    per_layer = (zs < height).sum(axis=1) / float(SUB)  # x/y samples do not matter
    out = np.empty((nz, ny, nx), dtype=np.float64)
    out[:] = per_layer[:, None, None]
    return out


def random_drops(count: int = 32, seed: int = SEED_DROPS, film_top: float = 0.1,
                 rmin: float = 0.02, rmax: float = 0.06) -> List[Tuple[float, float, float, float]]:
    """Non-overlapping random drops above a film: list of (r, cx, cy, cz).

    Each candidate draws r ~ U[rmin,rmax], then cx, cy ~ U[r, 1-r] and
    cz ~ U[film_top + r, 1 - r], in that order; a candidate closer than the sum
    of radii to an accepted drop is rejected and redrawn.
    """
    rng = np.random.default_rng(seed)
    drops: List[Tuple[float, float, float, float]] = []
    tries = 0
    while len(drops) < count:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place drops")
        r = rng.uniform(rmin, rmax)
        cx = rng.uniform(r, 1.0 - r)
        cy = rng.uniform(r, 1.0 - r)
        cz = rng.uniform(film_top + r, 1.0 - r)
        ok = True
        for (r2, x2, y2, z2) in drops:
            if (cx - x2) ** 2 + (cy - y2) ** 2 + (cz - z2) ** 2 < (r + r2) ** 2:
                ok = False
                break
        if ok:
            drops.append((float(r), float(cx), float(cy), float(cz)))
    return drops


def velocity(dims: Sequence[int], seed: int = SEED_VELOCITY
             ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Face velocities u, v, w ~ U[-1, 1] (drawn in that order), boundary normals zeroed."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(nz, ny, nx + 1))
    v = rng.uniform(-1.0, 1.0, size=(nz, ny + 1, nx))
    w = rng.uniform(-1.0, 1.0, size=(nz + 1, ny, nx))
    u[:, :, 0] = 0.0
    u[:, :, nx] = 0.0
    v[:, 0, :] = 0.0
    v[:, ny, :] = 0.0
    w[0, :, :] = 0.0
    w[nz, :, :] = 0.0
    return u, v, w


def loss_weights(dims: Sequence[int], seed: int = SEED_WEIGHTS) -> np.ndarray:
    nx, ny, nz = dims
    return np.random.default_rng(seed).standard_normal((nz, ny, nx))


@dataclasses.dataclass
class Workload:
    """Raw inputs of one solve: VOF fractions, phase densities, velocity, spacing."""
    name: str
    dims: Tuple[int, int, int]          # (nx, ny, nz)
    f_drop: np.ndarray                  # [nz, ny, nx]
    f_film: np.ndarray                  # [nz, ny, nx]
    rho_drop: float = RHO_DROP
    rho_film: float = RHO_FILM
    rho_gas: float = RHO_GAS
    dt: float = 1.0
    u: Optional[np.ndarray] = None
    v: Optional[np.ndarray] = None
    w: Optional[np.ndarray] = None

    @property
    def h(self) -> float:
        return 1.0 / self.dims[0]


def _with_velocity(wl: Workload, seed: int, with_velocity: bool) -> Workload:
    if with_velocity:
        wl.u, wl.v, wl.w = velocity(wl.dims, seed)
    return wl


def sphere_workload(n: int = 32, seed: int = SEED_VELOCITY, with_velocity: bool = True) -> Workload:
    """Sphere r = 0.25 at the centre (drop phase, 1000) in air; no film."""
    dims = (n, n, n)
    f_drop = sphere_fraction(dims, (0.5, 0.5, 0.5), 0.25)
    f_film = np.zeros_like(f_drop)
    return _with_velocity(Workload("sphere", dims, f_drop, f_film), seed, with_velocity)


def drop_film_workload(n: int = 128, seed: int = SEED_VELOCITY, with_velocity: bool = True) -> Workload:
    """Film z < 0.15 (960) and a drop r = 0.12 at (0.5, 0.5, 0.35) (1000) in air."""
    dims = (n, n, n)
    f_film = film_fraction(dims, 0.15)
    f_drop = sphere_fraction(dims, (0.5, 0.5, 0.35), 0.12)
    return _with_velocity(Workload("drop_film", dims, f_drop, f_film), seed, with_velocity)


def spheroid_film_workload(n: int = 256, seed: int = SEED_VELOCITY, with_velocity: bool = True) -> Workload:
    """Film z < 0.15 and an oblate spheroid (0.15, 0.15, 0.08) at (0.5, 0.5, 0.23), tangent to it."""
    dims = (n, n, n)
    f_film = film_fraction(dims, 0.15)
    f_drop = ellipsoid_fraction(dims, (0.5, 0.5, 0.23), (0.15, 0.15, 0.08))
    return _with_velocity(Workload("spheroid_film", dims, f_drop, f_film), seed, with_velocity)


def many_drops_workload(n: int = 512, seed: int = SEED_VELOCITY, drop_seed: int = SEED_DROPS,
                        count: int = 32, with_velocity: bool = True) -> Workload:
    """Film z < 0.1 (960) and 32 random non-overlapping drops (1000) in air."""
    dims = (n, n, n)
    f_film = film_fraction(dims, 0.1)
    f_drop = np.zeros((n, n, n), dtype=np.float64)
    for (r, cx, cy, cz) in random_drops(count, drop_seed, film_top=0.1):
        sphere_fraction(dims, (cx, cy, cz), r, out=f_drop)
    return _with_velocity(Workload("many_drops", dims, f_drop, f_film), seed, with_velocity)


def layered_film_workload(dims: Sequence[int], height: float = 0.15, seed: int = SEED_VELOCITY,
                          with_velocity: bool = False) -> Workload:
    """Film only (density varies in z alone): the case with an exact tridiagonal reduction."""
    dims = tuple(int(d) for d in dims)
    f_film = film_fraction(dims, height)
    f_drop = np.zeros_like(f_film)
    return _with_velocity(Workload("layered_film", dims, f_drop, f_film), seed, with_velocity)


WORKLOADS = {
    "sphere": sphere_workload,
    "drop_film": drop_film_workload,
    "spheroid_film": spheroid_film_workload,
    "many_drops": many_drops_workload,
}

# The five configurations: name -> (workload generator, N, mode)
CONFIGS = {
    "sphere32_fp64": ("sphere", 32, "fp64"),
    "drop_film128_fp64": ("drop_film", 128, "fp64"),
    "spheroid_film256_mixed": ("spheroid_film", 256, "mixed"),
    "many_drops512_mixed": ("many_drops", 512, "mixed"),
    "drop_film256_adjoint": ("drop_film", 256, "adjoint"),
}


def make(name: str, n: Optional[int] = None, **kw) -> Workload:
    return WORKLOADS[name](n, **kw) if n is not None else WORKLOADS[name](**kw)
