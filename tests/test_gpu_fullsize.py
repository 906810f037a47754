"""Parity at the benchmark's full size and launch configuration (512^3, the film +
32 drops workload), at the 128^3 drop-film FP64 configuration and at the 256^3
mixed-precision configuration.

At 512^3 the oracle runs single kernels over the whole grid (a pass takes about
a second on the host cores), recomputes the residual of the GPU solutions, and
supplies sampled values of its own solutions stopped at relative residuals of
1e-10 and 1e-12 (tests/golden/<layout><N>_oracle.txt, written by
make_oracle_samples.py).
The exact z-layered solution (tridiagonal reduction, the real 960/1.2 density
jump) is checked at 512^3 as a property that holds at any size.

Whole-field parity at 512^3: the oracle solves the film + 32 drops workload
inline (FP64 V-cycles, stopped at rr 1e-10 by the same rule as the GPU, then
continued to rr 1e-13), and every GPU solve of the benchmark's configuration is
compared with it over all 134M cells.  The differentiable configuration (the
drop-film field at 256^3, loss sum(w p), adjoint to 1e-10) is compared with
the oracle's gradients over every cell and face.
"""
import os
import time

import numpy as np
import pytest
import torch

import oracle
import refs
from gpu_util import N, T, gpu_inputs, max_rel, note, oracle_inputs, rel_l2
from paper_2605_30082_amd import workloads as W

pytestmark = pytest.mark.gpu

S = pytest.importorskip("paper_2605_30082_amd.solver")

GOLDEN_DIR = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def big():
    note("building the 512^3 film + 32 drops workload")
    wl = W.many_drops_workload(512)
    gb, gd = gpu_inputs(wl)
    ob, od = oracle_inputs(wl)
    del wl.u, wl.v, wl.w
    return wl, gb, gd, ob, od


@pytest.fixture(scope="module")
def big_oracle(big):
    """The oracle's solutions of the 512^3 workload: stopped by the GPU's rule at
    rr 1e-10, and continued from there to rr 1e-13 (the converged solution)."""
    wl, gb, gd, ob, od = big
    t0 = time.time()
    r10 = oracle.solve(ob, od, wl.h, tol=1e-10)
    note(f"oracle 512^3 to rr 1e-10: {r10.cycles} cycles, rr {r10.rel_res:.3e}, {time.time() - t0:.1f} s")
    t0 = time.time()
    r13 = oracle.solve(ob, od, wl.h, tol=1e-13, p0=r10.p)
    note(f"oracle 512^3 continued to rr 1e-13: {r13.cycles} more cycles, rr {r13.rel_res:.3e}, "
         f"{time.time() - t0:.1f} s")
    return r10, r13


def true_rr(ob, od, p, h):
    b = od - od.mean()
    return float(np.linalg.norm(oracle.residual(ob, b, p, h)) / np.linalg.norm(b))


def read_golden(name="many_drops512"):
    meta, rows = {}, []
    with open(os.path.join(GOLDEN_DIR, f"{name}_oracle.txt")) as f:
        for line in f:
            if line.startswith("#"):
                parts = line[1:].split()
                if len(parts) == 2:
                    try:
                        meta[parts[0]] = float(parts[1])
                    except ValueError:
                        pass
                continue
            rows.append(line.split())
    idx = np.array([int(r[0]) for r in rows])
    val = {"tol10": np.array([float(r[1]) for r in rows]),
           "tol12": np.array([float(r[2]) for r in rows])}
    return meta, idx, val


def test_inputs_bitexact_512(big):
    wl, gb, gd, ob, od = big
    for a, r in zip(gb, ob):
        assert np.array_equal(N(a), r)
    assert np.array_equal(N(gd), od)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_single_kernels_512(big, precision):
    wl, gb, gd, ob, od = big
    note(f"512^3 single kernels {precision}")
    s = S.Solver(*gb, wl.h, precision=precision)
    g = np.random.default_rng(21)
    p = g.standard_normal(od.shape)
    tol = 1e-13 if precision == "fp64" else 2e-6
    for order in (0, 1):
        got = N(s.smooth(gd, T(p), level=0, sweeps=1, order=order, precision=precision))
        ref = p
        for c in ((0, 1) if order == 0 else (1, 0)):
            ref = oracle.rbgs_half(ob, od, ref, wl.h, c)
        assert max_rel(got, ref) < tol, (order, max_rel(got, ref))
        # two sweeps: one launch of the two-sweep kernel in FP32
        got = N(s.smooth(gd, T(p), level=0, sweeps=2, order=order, precision=precision))
        for c in ((0, 1) if order == 0 else (1, 0)):
            ref = oracle.rbgs_half(ob, od, ref, wl.h, c)
        assert max_rel(got, ref) < tol, (order, "2 sweeps", max_rel(got, ref))
    got = N(s.residual_restrict(gd, T(p), level=0, precision=precision))
    ref = oracle.restrict(oracle.residual(ob, od, p, wl.h))
    assert max_rel(got, ref) < tol * 10
    # the V-cycle's pre-smoothing from zero and the restriction of its residual
    # (FP32: one launch of the fused kernel, as the benchmark's V-cycles run it)
    pz, bc = s.presmooth_restrict(gd, level=0, precision=precision)
    pz = N(pz)
    ref = np.zeros_like(p)
    for c in (0, 1, 0, 1):
        ref = oracle.rbgs_half(ob, od, ref, wl.h, c)
    assert max_rel(pz, ref) < tol, ("presmooth", max_rel(pz, ref))
    ref = oracle.restrict(oracle.residual(ob, od, pz, wl.h))
    assert max_rel(N(bc), ref) < tol * 10, ("restrict", max_rel(N(bc), ref))
    e = g.standard_normal((256, 256, 256))
    got = N(s.prolong_correct(T(e), T(p), level=0, precision=precision))
    assert max_rel(got, oracle.prolong_add(e, p)) < tol
    s.close()


def test_solves_512(big):
    wl, gb, gd, ob, od = big
    meta, idx, val = read_golden()
    results = {}
    for precision in ("fp64", "mixed"):
        s = S.Solver(*gb, wl.h, precision=precision, zero_guess=True)
        p, st = s.solve(gd, 1e-10)
        pg = N(p)
        rr = true_rr(ob, od, pg, wl.h)
        note(f"512^3 {precision}: cycles {st.cycles} rr {st.rel_res:.3e} (oracle-recomputed {rr:.3e})")
        assert st.rel_res <= 1e-10
        assert rr <= 1.000001e-10
        assert abs(pg.mean()) <= 1e-14 * np.abs(pg).max()
        results[precision] = (pg, st)
        s.close()
    assert rel_l2(results["mixed"][0], results["fp64"][0]) < 1e-9
    # sampled comparison with the oracle stopped by the same rule after the same
    # number of V-cycles: the FP64 path differs only in rounding order
    rms = meta["tol10_norm2"] / np.sqrt(512 ** 3)
    for precision, (pg, st) in results.items():
        assert st.cycles == meta["tol10_cycles"]
        d = pg.ravel()[idx] - val["tol10"]
        sampled_rel = float(np.sqrt(np.mean(d ** 2)) / rms)
        worst = float(np.abs(d).max() / rms)
        note(f"  {precision} vs oracle (same rule): sampled rel {sampled_rel:.3e}, max {worst:.3e}")
        bound = 1e-11 if precision == "fp64" else 1e-9
        assert sampled_rel < bound and worst < 10 * bound
        assert abs(np.linalg.norm(pg) - meta["tol10_norm2"]) < bound * meta["tol10_norm2"]
    # a tighter GPU solve against the oracle's converged solution
    s = S.Solver(*gb, wl.h, precision="fp64", zero_guess=True)
    p, st = s.solve(gd, 1e-12)
    d = N(p).ravel()[idx] - val["tol12"]
    rms = meta["tol12_norm2"] / np.sqrt(512 ** 3)
    note(f"  fp64 tol 1e-12 ({st.cycles} cycles) vs converged oracle: "
         f"sampled rel {np.sqrt(np.mean(d ** 2)) / rms:.3e}, max {np.abs(d).max() / rms:.3e}")
    assert st.cycles == meta["tol12_cycles"]
    assert np.sqrt(np.mean(d ** 2)) < 1e-11 * rms and np.abs(d).max() < 1e-10 * rms
    s.close()


def test_density_context_512(big):
    """The benchmark's default configuration: the hierarchy built from the cell
    density.  Its solves equal the face-array solves bit for bit, in both precisions."""
    wl, gb, gd, ob, od = big
    meta, idx, val = read_golden()
    rho = S.density_from_vof(T(wl.f_drop), T(wl.f_film), wl.rho_drop, wl.rho_film, wl.rho_gas)
    for precision in ("mixed", "fp64"):
        kw = dict(precision=precision, zero_guess=True)
        with S.Solver.from_density(rho, wl.h, **kw) as s:
            pd, std = s.solve(gd, 1e-10)
        with S.Solver(*gb, wl.h, **kw) as s:
            pf, stf = s.solve(gd, 1e-10)
        note(f"512^3 density context {precision}: cycles {std.cycles} rr {std.rel_res:.3e}")
        assert torch.equal(pd, pf) and std.hist == stf.hist
        assert std.cycles == meta["tol10_cycles"] and std.rel_res <= 1e-10
        d = N(pd).ravel()[idx] - val["tol10"]
        rms = meta["tol10_norm2"] / np.sqrt(512 ** 3)
        assert np.sqrt(np.mean(d ** 2)) < (1e-11 if precision == "fp64" else 1e-9) * rms
        del pd, pf


def test_layered_film_512_exact():
    n = 512
    dims = (n, n, n)
    wl = W.layered_film_workload(dims, height=0.1)
    f = wl.f_film[:, 0, 0]
    rho = W.RHO_FILM * f + W.RHO_GAS * (1.0 - f)
    g = np.random.default_rng(22).standard_normal(n)
    rhs, p_ref = refs.layered_solve(dims, 1.0 / n, rho, 1, 2, g)
    gb = S.faces_from_vof(T(wl.f_drop), T(wl.f_film), wl.rho_drop, wl.rho_film, wl.rho_gas)
    for precision in ("fp64", "mixed"):
        s = S.Solver(*gb, 1.0 / n, precision=precision, zero_guess=True)
        p, st = s.solve(T(rhs), 1e-10)
        err = rel_l2(N(p), p_ref)
        note(f"layered 512^3 {precision}: cycles {st.cycles} rel err vs exact {err:.3e}")
        assert err < 1e-9
        s.close()


def test_spheroid_film_256_mixed():
    wl = W.spheroid_film_workload(256)
    gb, gd = gpu_inputs(wl)
    ob, od = oracle_inputs(wl)
    exact = oracle.solve(ob, od, wl.h, tol=1e-12).p
    meta, idx, val = read_golden("spheroid_film256")
    # the stored samples are the solution computed here
    assert max_rel(exact.ravel()[idx], val["tol12"]) < 1e-12
    out = {}
    for precision in ("fp64", "mixed"):
        s = S.Solver(*gb, wl.h, precision=precision, zero_guess=True)
        p, st = s.solve(gd, 1e-10)
        out[precision] = N(p)
        err = rel_l2(out[precision], exact)
        note(f"spheroid 256^3 {precision}: cycles {st.cycles} rel err {err:.3e}")
        assert err < 1e-9
        assert true_rr(ob, od, out[precision], wl.h) <= 1.000001e-10
        assert st.cycles == meta["tol10_cycles"]
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_drop_film_128_against_stored_oracle(precision):
    """The plain-FP64 configuration at 128^3 (and the mixed solve of it): the same
    number of V-cycles as the oracle under the same stopping rule, and its sampled
    solution to rounding order (FP64) or to the FP32 preconditioner's level (mixed)."""
    wl = W.drop_film_workload(128)
    gb, gd = gpu_inputs(wl)
    meta, idx, val = read_golden("drop_film128")
    with S.Solver(*gb, wl.h, precision=precision, zero_guess=True) as s:
        p, st = s.solve(gd, 1e-10)
    pg = N(p)
    rms = meta["tol10_norm2"] / np.sqrt(128 ** 3)
    d = pg.ravel()[idx] - val["tol10"]
    sampled = float(np.sqrt(np.mean(d ** 2)) / rms)
    note(f"drop film 128^3 {precision}: cycles {st.cycles} (oracle {meta['tol10_cycles']:.0f}), "
         f"sampled rel vs oracle {sampled:.3e}")
    assert st.cycles == meta["tol10_cycles"] and st.rel_res <= 1e-10
    bound = 1e-11 if precision == "fp64" else 1e-9
    assert sampled < bound and float(np.abs(d).max()) / rms < 10 * bound
    d12 = pg.ravel()[idx] - val["tol12"]
    assert float(np.sqrt(np.mean(d12 ** 2))) / rms < 1e-9


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_fcg_512(big, precision):
    wl, gb, gd, ob, od = big
    meta, idx, val = read_golden()
    s = S.Solver(*gb, wl.h, precision=precision, zero_guess=True, method="fcg")
    p, st = s.solve(gd, 1e-10)
    s.close()
    pg = N(p)
    rr = true_rr(ob, od, pg, wl.h)
    d = pg.ravel()[idx] - val["tol12"]
    rms = meta["tol12_norm2"] / np.sqrt(512 ** 3)
    sampled = float(np.sqrt(np.mean(d ** 2)) / rms)
    note(f"fcg 512^3 {precision}: iterations {st.cycles} rr {st.rel_res:.3e} (oracle-recomputed {rr:.3e}), "
         f"sampled rel vs converged oracle {sampled:.3e}")
    assert st.rel_res <= 1e-10 and rr <= 1.01e-10
    assert sampled < 1e-9


def test_largest_arrays_layered_exact():
    """1024 x 1024 x 256 cells: the FP64 face arrays exceed 2^31 bytes, so the FP64
    finest level runs the simple kernels (and the mixed outer update its simple form)
    while the FP32 V-cycle stays tiled.  Checked against the exact z-layered solution."""
    dims = (1024, 1024, 256)
    h = 1.0 / 1024
    wl = W.layered_film_workload(dims, height=0.1)
    f = wl.f_film[:, 0, 0]
    rho = W.RHO_FILM * f + W.RHO_GAS * (1.0 - f)
    g = np.random.default_rng(23).standard_normal(dims[2])
    rhs, p_ref = refs.layered_solve(dims, h, rho, 3, 1, g)
    gb = S.faces_from_vof(T(wl.f_drop), T(wl.f_film), wl.rho_drop, wl.rho_film, wl.rho_gas)
    del wl
    assert gb[0].numel() * 8 > 2 ** 31
    grhs = T(rhs)
    del rhs
    for precision in ("mixed", "fp64"):
        s = S.Solver(*gb, h, precision=precision, zero_guess=True)
        p, st = s.solve(grhs, 1e-10)
        err = rel_l2(N(p), p_ref)
        note(f"1024x1024x256 {precision}: cycles {st.cycles} rr {st.rel_res:.3e} rel err vs exact {err:.3e}")
        assert st.rel_res <= 1e-10 and err < 1e-9
        s.close()
        if precision == "mixed":
            # a density context of the same size: its 2 GiB density array is never
            # read by a tiled pass (they are off above 2^31 bytes); same solution
            rho_t = T(np.broadcast_to(rho[:, None, None], (dims[2], dims[1], dims[0])))
            with S.Solver.from_density(rho_t, h, precision=precision, zero_guess=True) as sd:
                pd, _ = sd.solve(grhs, 1e-10)
            assert torch.equal(pd, p)
            del pd, rho_t
        del p


@pytest.mark.parametrize("precision,method", [("mixed", "vcycle"), ("fp64", "vcycle"),
                                              ("mixed", "fcg"), ("fp64", "fcg")])
def test_whole_field_512_vs_oracle(big, big_oracle, precision, method):
    """The benchmark's configuration (hierarchy from the cell density, p = 0,
    rr 1e-10) against the oracle over all 134M cells: relative L2 <= 1e-9 from
    the converged solution; the V-cycle solves also against the oracle stopped
    by the same rule after the same number of cycles (FP64: rounding order
    only)."""
    wl, gb, gd, ob, od = big
    r10, r13 = big_oracle
    rho = S.density_from_vof(T(wl.f_drop), T(wl.f_film), wl.rho_drop, wl.rho_film, wl.rho_gas)
    with S.Solver.from_density(rho, wl.h, precision=precision, zero_guess=True, method=method) as s:
        p, st = s.solve(gd, 1e-10)
    del rho
    pg = N(p)
    del p
    err = rel_l2(pg, r13.p)
    note(f"512^3 {precision} {method}: {st.cycles} iterations, rr {st.rel_res:.3e}, "
         f"whole-field rel L2 vs converged oracle {err:.3e}")
    assert st.rel_res <= 1e-10
    assert err <= 1e-9
    if method == "vcycle":
        same = rel_l2(pg, r10.p)
        note(f"  vs the oracle stopped by the same rule ({r10.cycles} cycles): whole-field rel L2 {same:.3e}")
        assert st.cycles == r10.cycles
        assert same <= (1e-11 if precision == "fp64" else 1e-9)


@pytest.mark.parametrize("precision,persistent", [("fp64", False), ("mixed", True)])
def test_differentiable_drop_film_256(precision, persistent):
    """Loss = sum(w p), w ~ N(0, 1) (seed 2), on the drop-film field at 256^3: the
    forward and the adjoint solve to rr 1e-10 through the autograd function (a
    hierarchy per call, or one persistent Solver re-used by forward and backward),
    against the oracle's p, lambda = dLoss/drhs and dLoss/dbeta over every cell and
    interior face, and the adjoint's own residual recomputed by the oracle."""
    from paper_2605_30082_amd.autograd import poisson_solve
    wl = W.drop_film_workload(256)
    w = W.loss_weights(wl.dims)
    gb, gd = gpu_inputs(wl)
    ob, od = oracle_inputs(wl)
    rhs = gd.clone().requires_grad_(True)
    bx, by, bz = (a.clone().requires_grad_(True) for a in gb)
    solver = S.Solver(*gb, wl.h, precision=precision, zero_guess=True) if persistent else None
    t0 = time.time()
    p = poisson_solve(rhs, bx, by, bz, wl.h, tol=1e-10, precision=precision, solver=solver)
    (T(w) * p).sum().backward()
    torch.cuda.synchronize()
    note(f"drop film 256^3 {precision} autograd (persistent solver: {persistent}): "
         f"forward + backward {time.time() - t0:.2f} s")
    if solver is not None:
        solver.close()
    t0 = time.time()
    p_o, lam_o, g_o = oracle.gradients(ob, od, w, wl.h, tol=1e-13)
    note(f"  oracle gradients {time.time() - t0:.1f} s")
    lam = N(rhs.grad)
    wz = w - w.mean()
    adj_rr = float(np.linalg.norm(oracle.residual(ob, wz, lam, wl.h)) / np.linalg.norm(wz))
    e_p, e_lam = rel_l2(N(p), p_o), rel_l2(lam, lam_o)
    e_g = [rel_l2(N(a), r) for a, r in zip((bx.grad, by.grad, bz.grad), g_o)]
    note(f"  rel L2: p {e_p:.3e}, lambda {e_lam:.3e}, g_beta {max(e_g):.3e}; adjoint rr {adj_rr:.3e}")
    assert adj_rr <= 1.000001e-10
    assert e_p <= 1e-9 and e_lam <= 1e-9
    assert max(e_g) <= 1e-8
    gx, gy, gz = (N(a) for a in (bx.grad, by.grad, bz.grad))
    assert not gx[:, :, [0, -1]].any() and not gy[:, [0, -1], :].any() and not gz[[0, -1]].any()
