"""Contexts built from a cell density (mg_setup_density) against contexts built
from face arrays, and both against the oracle.

The density context forms the finest-grid FP64 coefficients 2/(rho_L + rho_R)
inside the residual passes instead of reading them; the quotient is the one
that defines the face arrays, so every result must be identical bit for bit:
single kernels, V-cycle and flexible-CG solves, in both precisions, on grids
that span several 64 x 32 tiles with a ragged last tile."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import N, T, max_rel, note
from paper_2605_30082_amd import workloads as W

pytestmark = pytest.mark.gpu

S = pytest.importorskip("paper_2605_30082_amd.solver")

DIMS = [(64, 48, 32), (96, 64, 32), (128, 64, 64), (192, 128, 64)]


def random_density(dims, seed):
    """Cells of the three phases (gas 1.2, film 960, drop 1000) in random blocks,
    with fractional mixtures on a quarter of the cells: density jumps of 800x
    between neighbours, as at a liquid-gas interface."""
    nx, ny, nz = dims
    g = np.random.default_rng(seed)
    phase = g.choice(np.array([W.RHO_GAS, W.RHO_FILM, W.RHO_DROP]), size=(nz // 4, ny // 4, nx // 4))
    rho = np.repeat(np.repeat(np.repeat(phase, 4, 0), 4, 1), 4, 2).copy()
    mix = g.random(rho.shape) < 0.25
    f = g.random(rho.shape)
    rho[mix] = W.RHO_DROP * f[mix] + W.RHO_GAS * (1.0 - f[mix])
    return rho


def drops_density(dims, seed):
    """A film (z < 0.2 of the height) and four seeded drops in air, fractions by
    sub-cell sampling: the structure of the benchmark workloads on any grid."""
    g = np.random.default_rng(seed)
    film = W.film_fraction(dims, 0.2)
    drop = np.zeros_like(film)
    for _ in range(4):
        r = g.uniform(0.08, 0.15)
        W.sphere_fraction(dims, (g.uniform(r, 1 - r), g.uniform(r, 1 - r), g.uniform(0.2 + r, 1 - r)), r, drop)
    drop = np.minimum(drop, 1.0)
    gas = np.maximum(1.0 - drop - film, 0.0)
    return W.RHO_DROP * drop + W.RHO_FILM * film + W.RHO_GAS * gas


def inputs(dims, seed, smooth=False):
    g = np.random.default_rng(seed + 100)
    nx, ny, nz = dims
    rho = drops_density(dims, seed) if smooth else random_density(dims, seed)
    return rho, g.standard_normal((nz, ny, nx)), g.standard_normal((nz, ny, nx))


@pytest.mark.parametrize("make,n", [(W.sphere_workload, 32), (W.drop_film_workload, 64)])
def test_density_and_faces_bitexact(make, n):
    wl = make(n, with_velocity=False)
    args = (wl.rho_drop, wl.rho_film, wl.rho_gas)
    rho = S.density_from_vof(T(wl.f_drop), T(wl.f_film), *args)
    orho = oracle.density(wl.f_drop, wl.f_film, *args)
    assert np.array_equal(N(rho), orho)
    from_rho = S.faces_from_density(rho)
    from_vof = S.faces_from_vof(T(wl.f_drop), T(wl.f_film), *args)
    ref = oracle.face_coeffs(orho)
    for a, b, r in zip(from_rho, from_vof, ref):
        assert np.array_equal(N(a), N(b))
        assert np.array_equal(N(a), r)


@pytest.mark.parametrize("dims", DIMS)
def test_density_context_kernels_identical(dims):
    rho, b, p = inputs(dims, 1)
    h = 1.0 / dims[0]
    sd = S.Solver.from_density(T(rho), h, precision="mixed")
    sf = S.Solver(*S.faces_from_density(T(rho)), h, precision="mixed")
    assert sd.num_levels == sf.num_levels
    for level in range(sd.num_levels):
        for a, c in zip(sd.level_faces(level), sf.level_faces(level)):
            assert torch.equal(a, c)
    for precision in ("fp64", "mixed"):
        got = sd.residual_restrict(T(b), T(p), level=0, precision=precision)
        assert torch.equal(got, sf.residual_restrict(T(b), T(p), level=0, precision=precision))
        for order in (0, 1):
            for sweeps in (1, 2):
                got = sd.smooth(T(b), T(p), level=0, sweeps=sweeps, order=order, precision=precision)
                ref = sf.smooth(T(b), T(p), level=0, sweeps=sweeps, order=order, precision=precision)
                assert torch.equal(got, ref), (precision, order, sweeps)
    assert sd.residual_norm2(T(b), T(p)) == sf.residual_norm2(T(b), T(p))
    # the density kernels against the oracle's definition
    ob = oracle.face_coeffs(rho)
    r = oracle.residual(ob, b, p, h)
    got = N(sd.residual_restrict(T(b), T(p), level=0, precision="fp64"))
    assert max_rel(got, oracle.restrict(r)) < 1e-13
    n2 = sd.residual_norm2(T(b), T(p))
    assert abs(n2 - float(np.sum(r * r))) <= 1e-12 * float(np.sum(r * r))
    ref = p
    for colour in (0, 1):
        ref = oracle.rbgs_half(ob, b, ref, h, colour)
    got = N(sd.smooth(T(b), T(p), level=0, sweeps=1, order=0, precision="fp64"))
    assert max_rel(got, ref) < 1e-13
    sd.close()
    sf.close()


@pytest.mark.parametrize("method", ["vcycle", "fcg"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("dims", [(32, 16, 24)] + DIMS[:3])
def test_density_context_solves_identical(dims, precision, method):
    """(32, 16, 24): no level is wide enough for the tiled kernels, so the density
    context runs the simple kernels on its stored faces throughout."""
    rho, b, _ = inputs(dims, 2, smooth=True)
    h = 1.0 / dims[0]
    kw = dict(precision=precision, zero_guess=True, method=method)
    out = []
    for s in (S.Solver.from_density(T(rho), h, **kw), S.Solver(*S.faces_from_density(T(rho)), h, **kw)):
        p, st = s.solve(T(b), 1e-10)
        out.append((p, st))
        s.close()
    (pd, sd), (pf, sf) = out
    note(f"density context {dims} {precision} {method}: cycles {sd.cycles} rr {sd.rel_res:.3e}")
    assert torch.equal(pd, pf)
    assert sd.cycles == sf.cycles and sd.hist == sf.hist
    ob = oracle.face_coeffs(rho)
    bb = b - b.mean()
    rr = np.linalg.norm(oracle.residual(ob, bb, N(pd), h)) / np.linalg.norm(bb)
    assert sd.rel_res <= 1e-10 and rr <= 1.01e-10


def test_density_update_switch_and_rejects():
    dims = (64, 32, 48)
    h = 1.0 / 64
    rho1, b, _ = inputs(dims, 3, smooth=True)
    rho2 = drops_density(dims, 4)
    kw = dict(precision="mixed", zero_guess=True)

    def face_solve(rho):
        with S.Solver(*S.faces_from_density(T(rho)), h, **kw) as s:
            return s.solve(T(b), 1e-10)[0]

    ref1, ref2 = face_solve(rho1), face_solve(rho2)
    s = S.Solver.from_density(T(rho1), h, **kw)
    assert torch.equal(s.solve(T(b), 1e-10)[0], ref1)
    s.update_density(T(rho2))
    assert torch.equal(s.solve(T(b), 1e-10)[0], ref2)
    s.update(*S.faces_from_density(T(rho1)))          # back to face arrays
    assert torch.equal(s.solve(T(b), 1e-10)[0], ref1)
    s.update_density(T(rho2))                         # and to the density again
    assert torch.equal(s.solve(T(b), 1e-10)[0], ref2)
    for bad_value in (-1.0, 0.0, float("nan"), float("inf")):
        bad = rho2.copy()
        bad[5, 6, 7] = bad_value
        with pytest.raises(S.MgError) as e:
            s.update_density(T(bad))
        assert e.value.status == S.L.MG_EINVAL and "density" in str(e.value)
        with pytest.raises(S.MgError):               # rejected coefficients block solves
            s.solve(T(b), 1e-10)
        with pytest.raises(S.MgError):
            S.Solver.from_density(T(bad), h, **kw)
    s.update_density(T(rho1))
    assert torch.equal(s.solve(T(b), 1e-10)[0], ref1)
    s.close()
    with S.Solver(*S.faces_from_density(T(rho1)), h, **kw) as f:
        with pytest.raises(S.MgError) as e:
            f.update_density(T(rho1))
        assert "mg_setup_density" in str(e.value)
