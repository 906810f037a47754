"""The solve that allocates nothing (mg_solve_noalloc, static per-GPU scratch)
against the allocating entry points (mg_setup + mg_solve) on the same
arguments: identical solutions, cycle counts and residual histories, on two
calls in a row where the second has a smaller grid (the scratch keeps the first
call's contents), in both precisions and for both iterations.  Sizes beyond the
scratch, and timing (which needs events), are refused before any device work.

Collected last: a failure here cannot hide the other GPU tests."""
import numpy as np
import pytest
import torch

from gpu_util import T, gpu_inputs
from paper_2605_30082_amd import _lib as L
from paper_2605_30082_amd import workloads as W

pytestmark = pytest.mark.gpu

S = pytest.importorskip("paper_2605_30082_amd.solver")


def reference(gb, gd, h, **kw):
    with S.Solver(*gb, h, zero_guess=True, **kw) as s:
        return s.solve(gd, 1e-10)


@pytest.mark.parametrize("precision,method", [("fp64", "vcycle"), ("mixed", "vcycle"), ("mixed", "fcg"),
                                              ("fp64", "fcg")])
def test_noalloc_matches_allocating_solve(precision, method):
    # 64^3 drop on a film (every tiled kernel), then a smaller 32^3 sphere
    for wl in (W.drop_film_workload(64), W.sphere_workload(32)):
        gb, gd = gpu_inputs(wl)
        p_ref, st_ref = reference(gb, gd, wl.h, precision=precision, method=method)
        p = torch.full_like(gd, 7.0)            # ignored: zero_guess
        st = S.solve_noalloc(*gb, wl.h, gd, p, 1e-10, precision=precision, method=method, zero_guess=True)
        torch.cuda.synchronize()
        assert st.status == L.MG_OK and st.rel_res <= 1e-10
        assert st.cycles == st_ref.cycles and st.hist == st_ref.hist, (wl.name, st.hist, st_ref.hist)
        assert torch.equal(p, p_ref), (wl.name, float((p - p_ref).abs().max()))


def test_noalloc_warm_start_and_level_launches():
    wl = W.drop_film_workload(64)
    gb, gd = gpu_inputs(wl)
    g = np.random.default_rng(5)
    p0 = T(g.standard_normal(gd.shape))
    for kw in (dict(precision="fp64"), dict(precision="mixed", level_launches=True)):
        with S.Solver(*gb, wl.h, **kw) as s:
            p_ref, st_ref = s.solve(gd, 1e-10, p=p0.clone())
        p = p0.clone()
        st = S.solve_noalloc(*gb, wl.h, gd, p, 1e-10, **kw)
        assert st.cycles == st_ref.cycles and torch.equal(p, p_ref)


def test_noalloc_refuses_grids_beyond_the_scratch_and_timing():
    import ctypes
    lib = L.load()
    dev = torch.device("cuda", 0)
    n = 128                                     # 128^3 FP64 needs more than the scratch holds
    shapes = S.face_shapes((n, n, n))
    beta = [torch.ones(s, dtype=torch.float64, device=dev) for s in shapes]
    rhs = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    p = torch.zeros_like(rhs)
    with pytest.raises(L.MgError) as e:
        S.solve_noalloc(*beta, 1.0 / n, rhs, p, 1e-10)
    assert e.value.status == L.MG_EINVAL and "no-allocation buffer" in str(e.value)
    n = 16
    shapes = S.face_shapes((n, n, n))
    beta = [torch.ones(s, dtype=torch.float64, device=dev) for s in shapes]
    rhs = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    p = torch.zeros_like(rhs)
    opts = L.MgOpts(2, 2, 100, 4, L.MG_PREC_FP64, L.MG_FLAG_TIMING)
    st = lib.mg_solve_noalloc(*[ctypes.c_void_p(a.data_ptr()) for a in beta], L.dims_arg((n, n, n)), 1.0 / n,
                              L.MG_BC_NEUMANN, ctypes.byref(opts), ctypes.c_void_p(rhs.data_ptr()),
                              ctypes.c_void_p(p.data_ptr()), 1e-10, None, None)
    assert st == L.MG_EINVAL and "MG_FLAG_TIMING" in L.last_error(None)
