"""Edge cases of the GPU solver against the oracle: degenerate and single-level
grids, ragged and anisotropic grids, warm starts, coefficient updates, and the
argument checks of the Python front end."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import N, T, dev, gpu_inputs, note, oracle_inputs, rel_l2
from paper_2605_30082_amd import workloads as W

pytestmark = pytest.mark.gpu

S = pytest.importorskip("paper_2605_30082_amd.solver")


def random_beta(dims, seed):
    nx, ny, nz = dims
    g = np.random.default_rng(seed)
    return (g.uniform(1e-3, 0.9, (nz, ny, nx + 1)), g.uniform(1e-3, 0.9, (nz, ny + 1, nx)),
            g.uniform(1e-3, 0.9, (nz + 1, ny, nx)))


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 1), (1, 3, 2), (4, 4, 4), (3, 3, 3), (8, 8, 8),
                                  (96, 96, 96), (128, 64, 32), (16, 32, 64), (64, 64, 16)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_on_unusual_grids(dims, precision):
    nx, ny, nz = dims
    beta = random_beta(dims, 31)
    h = 1.0 / max(dims)
    rhs = np.random.default_rng(32).standard_normal((nz, ny, nx))
    s = S.Solver(T(beta[0]), T(beta[1]), T(beta[2]), h, precision=precision, zero_guess=True)
    p, st = s.solve(T(rhs), 1e-10)
    pg = N(p)
    ref = oracle.solve(beta, rhs, h, tol=1e-13)
    note(f"{dims} {precision}: levels {s.num_levels} cycles {st.cycles} (oracle {ref.cycles})")
    if rhs.size == 1:
        assert st.cycles == 0 and np.all(pg == 0)
    else:
        assert st.rel_res <= 1e-10
        assert rel_l2(pg, ref.p) < 1e-9
    s.close()


# 64^3 takes the FP64 path whose residual norm comes from the sweep that starts
# the next cycle; 32^3 the separate norm pass
@pytest.mark.parametrize("n", [32, 64])
def test_warm_start_matches_oracle_lockstep(n):
    wl = W.drop_film_workload(n)
    gb, gd = gpu_inputs(wl)
    ob, od = oracle_inputs(wl)
    p0 = np.random.default_rng(33).standard_normal(od.shape)
    s = S.Solver(*gb, wl.h, max_cycles=3)
    p, st = s.solve(gd, 1e-14, p=T(p0), check=False)
    ref = oracle.solve(ob, od, wl.h, tol=1e-14, max_cycles=3, p0=p0, check=False)
    assert st.status == S.L.MG_ENOCONV and ref.status == oracle.OR_ENOCONV
    np.testing.assert_allclose(st.hist, ref.hist, rtol=1e-8)
    assert rel_l2(N(p), ref.p) < 1e-11
    s.close()


def test_update_equals_fresh_setup():
    a = W.drop_film_workload(64)
    b = W.sphere_workload(64)
    ga, gda = gpu_inputs(a)
    gbb, gdb = gpu_inputs(b)
    s = S.Solver(*ga, a.h, precision="mixed", zero_guess=True)
    s.update(*gbb)
    p1, st1 = s.solve(gdb, 1e-10)
    s2 = S.Solver(*gbb, b.h, precision="mixed", zero_guess=True)
    p2, st2 = s2.solve(gdb, 1e-10)
    assert st1.cycles == st2.cycles
    assert torch.equal(p1, p2)
    # a rejected update leaves the context unusable until the next good update
    bad = gbb[0].clone()
    bad[5, 5, 5] = float("nan")
    with pytest.raises(S.MgError):
        s.update(bad, gbb[1], gbb[2])
    with pytest.raises(S.MgError):
        s.solve(gdb, 1e-10)
    s.update(*ga)
    p3, _ = s.solve(gda, 1e-10)
    assert torch.isfinite(p3).all()
    s.close()
    s2.close()


def test_misaligned_p_is_rejected():
    wl = W.sphere_workload(8)
    gb, gd = gpu_inputs(wl)
    s = S.Solver(*gb, wl.h)
    buf = torch.zeros(8 * 8 * 8 + 1, dtype=torch.float64, device=dev())
    p = buf[1:].view(8, 8, 8)
    with pytest.raises(S.MgError) as ei:
        s.solve(gd, 1e-10, p=p)
    assert "aligned" in str(ei.value)
    s.close()


def test_front_end_argument_checks():
    wl = W.sphere_workload(8)
    gb, gd = gpu_inputs(wl)
    with pytest.raises(TypeError):
        S.Solver(gb[0].float(), gb[1], gb[2], wl.h)
    with pytest.raises(ValueError):
        S.Solver(gb[0].cpu(), gb[1], gb[2], wl.h)
    with pytest.raises(S.MgError):
        S.Solver(*gb, wl.h, precision="half")
    with pytest.raises(S.MgError):
        S.Solver(*gb, wl.h, bc="dirichlet")
    s = S.Solver(*gb, wl.h)
    with pytest.raises(ValueError):
        s.solve(gd[:4].contiguous(), 1e-10)
    s.close()


@pytest.mark.parametrize("density", [False, True])
def test_kernel_timing_stats(density):
    """MG_FLAG_TIMING: every timed launch is counted with its event duration and
    algorithmic bytes, and timing does not change the result."""
    import paper_2605_30082_amd._lib as L
    wl = W.drop_film_workload(64)
    gb, gd = gpu_inputs(wl)
    rho = S.density_from_vof(T(wl.f_drop), T(wl.f_film), wl.rho_drop, wl.rho_film, wl.rho_gas)

    def make(**kw):
        return S.Solver.from_density(rho, wl.h, **kw) if density else S.Solver(*gb, wl.h, **kw)

    for precision in ("mixed", "fp64"):
        with make(precision=precision, zero_guess=True, timing=True) as s:
            p1, st = s.solve(gd, 1e-10)
        with make(precision=precision, zero_guess=True) as s:
            p0, st0 = s.solve(gd, 1e-10)
        assert torch.equal(p0, p1) and st.cycles == st0.cycles
        n = st.cycles
        if precision == "mixed":
            # at 64^3 only the finest grid is wide enough for the tiled kernels
            # (from p = 0 the initial residual is the rhs itself: no outer update before cycle 1;
            # the pre-smoothing launch also restricts the residual, the post-smoothing's
            # first two-sweep launch does the prolongation itself)
            expect = {L.MG_K_SWEEP2R: n, L.MG_K_SWEEP2: n, L.MG_K_RESTRICT: 0, L.MG_K_PROLONG: 0,
                      L.MG_K_OUTER: n}
        else:
            # pre- and post-smoothing each one two-sweep launch (the post-smoothing
            # one prolongates the coarse correction itself); the norm of each
            # cycle's result is a residual pass of its own
            expect = {L.MG_K_SWEEP2: 2 * n, L.MG_K_SWEEP: 0, L.MG_K_NORM: n, L.MG_K_RESTRICT: n,
                      L.MG_K_PROLONG: 0}
        # (mixed) the next cycle's pre-sweeps are queued while the host waits for a
        # norm; one such launch may run in vain after the last cycle
        spare = 1 if precision == "mixed" and st.kernel_launches[L.MG_K_SWEEP2R] == n + 1 else 0
        if spare:
            expect[L.MG_K_SWEEP2R] += 1
        for k, count in expect.items():
            assert st.kernel_launches[k] == count, (precision, k, st.kernel_launches[k], count)
            assert st.kernel_launches_finest[k] == count
            assert (st.kernel_ms[k] > 0 and st.kernel_bytes[k] > 0) == (count > 0)
            assert st.kernel_ms_finest[k] == st.kernel_ms[k]
        assert sum(st.kernel_ms) < st.solve_ms
        assert sum(st0.kernel_launches) == 0
        # a class mask: only the selected class is timed, results unchanged
        with make(precision=precision, zero_guess=True, timing=True) as s:
            only = L.MG_K_SWEEP2R if precision == "mixed" else L.MG_K_RESTRICT
            s.set_timing_classes([only])
            p2, st2 = s.solve(gd, 1e-10)
            assert torch.equal(p2, p0)
            assert st2.kernel_launches[only] == expect[only]
            assert sum(st2.kernel_launches) == expect[only]
            s.set_timing_classes(None)
            _, st3 = s.solve(gd, 1e-10)
            assert list(st3.kernel_launches) == list(st.kernel_launches)
            with pytest.raises(S.MgError):
                s.set_timing_classes([L.MG_K_COUNT])
    with make(precision="mixed") as s:
        with pytest.raises(S.MgError):
            s.set_timing_classes([0])


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 1), (1, 3, 2), (3, 3, 3), (8, 8, 8), (96, 96, 96),
                                  (128, 64, 32), (16, 32, 64), (64, 64, 16)])
def test_density_context_on_unusual_grids(dims):
    """Density contexts on single cells, one-cell-thick and ragged grids: identical to
    the face arrays mg_faces_from_density writes, in both precisions."""
    nx, ny, nz = dims
    g = np.random.default_rng(33)
    # a smooth density spanning 1.2 .. 1000 (sin product on the cell centres)
    zz, yy, xx = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx,
                             indexing="ij")
    s3 = np.sin(2 * np.pi * xx) * np.sin(2 * np.pi * yy) * np.sin(2 * np.pi * zz)
    rho = np.sqrt(1.2 * 1000.0) * np.exp(0.5 * np.log(1000.0 / 1.2) * s3)
    rhs = g.standard_normal((nz, ny, nx))
    h = 1.0 / max(dims)
    faces = S.faces_from_density(T(rho))
    for precision in ("fp64", "mixed"):
        kw = dict(precision=precision, zero_guess=True)
        with S.Solver.from_density(T(rho), h, **kw) as s:
            pd, std = s.solve(T(rhs), 1e-10)
        with S.Solver(*faces, h, **kw) as s:
            pf, stf = s.solve(T(rhs), 1e-10)
        assert torch.equal(pd, pf) and std.cycles == stf.cycles


@pytest.mark.parametrize("density", [False, True])
def test_mixed_zero_guess_without_cycles(density):
    """From p = 0 the mixed loop starts from the rhs itself; a tolerance the start
    already meets returns p = 0 whatever the caller's buffer held."""
    wl = W.drop_film_workload(64)
    gb, gd = gpu_inputs(wl)
    rho = S.density_from_vof(T(wl.f_drop), T(wl.f_film), wl.rho_drop, wl.rho_film, wl.rho_gas)
    kw = dict(precision="mixed", zero_guess=True)
    s = S.Solver.from_density(rho, wl.h, **kw) if density else S.Solver(*gb, wl.h, **kw)
    garbage = torch.randn(gd.shape, dtype=torch.float64, device=gd.device)
    p, st = s.solve(gd, 2.0, p=garbage)
    assert st.cycles == 0 and st.hist[0] == 1.0
    assert torch.count_nonzero(p) == 0
    # and a full solve from the same garbage buffer equals one from a zero buffer
    p1, st1 = s.solve(gd, 1e-10, p=torch.randn(gd.shape, dtype=torch.float64, device=gd.device))
    p2, st2 = s.solve(gd, 1e-10, p=torch.zeros_like(gd))
    assert torch.equal(p1, p2) and st1.hist == st2.hist
    s.close()


@pytest.mark.parametrize("dims", [(8, 8, 8), (16, 16, 16), (8, 16, 32), (12, 8, 16), (32, 32, 32), (96, 96, 96),
                                  (128, 64, 32), (64, 64, 16), (96, 96, 128)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("method", ["vcycle", "fcg"])
def test_fused_launches_match_level_launches(dims, precision, method):
    """By default the levels of at most 4096 cells run as one single-workgroup
    launch and (mixed) the pre-smoothing's two-sweep launch also restricts its
    residual and the post-smoothing's two-sweep launch prolongates the coarse
    correction itself; with level_launches=True every step is its own launch.
    Same values in the same order: identical solutions and histories.
    (96, 96, 128): ragged last x-tile and z-chunk of the pre-smoothing launch."""
    nx, ny, nz = dims
    beta = random_beta(dims, 41)
    h = 1.0 / max(dims)
    rhs = T(np.random.default_rng(42).standard_normal((nz, ny, nx)))
    out = []
    for level_launches in (False, True):
        with S.Solver(T(beta[0]), T(beta[1]), T(beta[2]), h, precision=precision, zero_guess=True,
                      method=method, level_launches=level_launches) as s:
            out.append(s.solve(rhs, 1e-10))
    (p0, st0), (p1, st1) = out
    note(f"{dims} {precision} {method}: cycles {st0.cycles}")
    assert st0.status == S.L.MG_OK and st0.rel_res <= 1e-10
    assert torch.equal(p0, p1) and st0.hist == st1.hist


@pytest.mark.parametrize("pre,post", [(0, 2), (3, 1), (1, 0), (2, 3)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_launches_sweep_counts(pre, post, precision):
    """Odd and zero sweep counts: the iterate changes buffers with every sweep
    and starts from a filled zero when no pre-sweep runs; warm starts too.
    128 x 32 x 32: the finest grid takes the two-sweep kernel (and its fused
    prolongation when post >= 2), 32 x 8 x 8 and below the single-workgroup launch."""
    dims = (128, 32, 32)
    nx, ny, nz = dims
    beta = random_beta(dims, 43)
    g = np.random.default_rng(44)
    rhs = T(g.standard_normal((nz, ny, nx)))
    p_start = g.standard_normal((nz, ny, nx))
    out = []
    for level_launches in (False, True):
        with S.Solver(T(beta[0]), T(beta[1]), T(beta[2]), 1.0 / 128, precision=precision, pre=pre, post=post,
                      max_cycles=6, level_launches=level_launches) as s:
            p, st = s.solve(rhs, 1e-14, p=T(p_start), check=False)
            out.append((p, st))
    (p0, st0), (p1, st1) = out
    assert st0.cycles == 6 and st0.hist == st1.hist
    assert torch.equal(p0, p1)


@pytest.mark.parametrize("method", ["vcycle", "fcg"])
def test_queued_presweeps_never_change_the_result(method):
    """The next cycle's pre-sweeps are queued while the host waits for a norm
    (not after the last allowed cycle, nor when the norm is expected to meet the
    tolerance).  Stopping after cycle k by the tolerance or by max_cycles takes
    different queueing decisions and must give the same p bit for bit."""
    wl = W.drop_film_workload(64)
    gb, gd = gpu_inputs(wl)
    kw = dict(precision="mixed", zero_guess=True, method=method)
    with S.Solver(*gb, wl.h, **kw) as s:
        _, full = s.solve(gd, 1e-13, check=False)
    for k in (3, 6, len(full.hist) - 2):
        tol = full.hist[k] * (1.0 + 1e-9)
        with S.Solver(*gb, wl.h, **kw) as s:
            p_tol, st_tol = s.solve(gd, tol)
        with S.Solver(*gb, wl.h, max_cycles=k, **kw) as s:
            p_max, st_max = s.solve(gd, 1e-30, check=False)
        assert st_tol.cycles == k and st_max.cycles == k
        assert st_tol.hist == st_max.hist == full.hist[:k + 1]
        assert torch.equal(p_tol, p_max)


@pytest.mark.parametrize("dims", [(1, 1, 1), (1, 5, 3), (70, 3, 130), (130, 9, 2), (64, 4, 64), (3, 200, 7)])
def test_face_passes_on_odd_shapes(dims):
    """The z-marching face kernels (coefficients from the VOF fractions or from
    a density; the face gradient): single cells and columns, a ragged last
    x-tile, fewer rows than a block, one-plane z-chunks, rows beyond one block:
    bit-exact with the oracle."""
    nx, ny, nz = dims
    note(f"face passes dims={dims}")
    g = np.random.default_rng(61)
    fd = g.uniform(0, 1, (nz, ny, nx))
    ff = g.uniform(0, 1, (nz, ny, nx)) * (1.0 - fd)
    gb = S.faces_from_vof(T(fd), T(ff), 1000.0, 960.0, 1.2)
    ob = oracle.faces_from_vof(fd, ff, 1000.0, 960.0, 1.2)
    for a, r in zip(gb, ob):
        np.testing.assert_array_equal(N(a), r)
    rho = oracle.density(fd, ff, 1000.0, 960.0, 1.2)
    for a, r in zip(S.faces_from_density(T(rho)), oracle.face_coeffs(rho)):
        np.testing.assert_array_equal(N(a), r)


@pytest.mark.parametrize("dims", [(1, 1, 1), (3, 3, 3), (12, 4, 8), (96, 32, 32), (4, 1, 2)])
def test_face_grad_on_odd_shapes(dims):
    """mg_face_grad on grids a context accepts, down to one cell: the oracle's
    (lambda_R - lambda_L)(p_R - p_L)/h^2 to the rounding of a division against
    a product with 1/h^2 (h = 1/96, 1/3, ... are not powers of 2), walls 0; a
    density context (faces formed by the same kernel, with its count of bad
    faces) equals a face context bit for bit."""
    nx, ny, nz = dims
    g = np.random.default_rng(62)
    rho = g.uniform(1.0, 1000.0, (nz, ny, nx))
    h = 1.0 / max(dims)
    lam, p = g.standard_normal((nz, ny, nx)), g.standard_normal((nz, ny, nx))
    with S.Solver(*[T(a) for a in oracle.face_coeffs(rho)], h) as s:
        got = s.face_grad(T(lam), T(p))
        for a, r in zip(got, oracle.face_grad(lam, p, h)):
            np.testing.assert_allclose(N(a), r, rtol=1e-15, atol=1e-300)
        faces = [N(a) for a in s.level_faces(0)]
    with S.Solver.from_density(T(rho), h) as sd:
        for a, r in zip(sd.level_faces(0), faces):
            np.testing.assert_array_equal(N(a), r)
