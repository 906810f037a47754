"""The stored sampled oracle solutions (tests/golden/<layout><N>_oracle.txt) are
what the oracle computes today: the 128^3 file is recomputed and compared value
for value, the larger ones are checked for structure and self-consistency.
The GPU tests and the benchmark read these files as the oracle's answer at sizes
where running the oracle inline would take minutes."""
import os

import numpy as np
import pytest

import oracle
from paper_2605_30082_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FILES = {("drop_film", 128), ("spheroid_film", 256), ("many_drops", 512)}


def read(layout, n):
    meta, rows = {}, []
    with open(os.path.join(GOLDEN, f"{layout}{n}_oracle.txt")) as f:
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
    return meta, idx, np.array([[float(r[1]), float(r[2])] for r in rows])


@pytest.mark.parametrize("layout,n", sorted(FILES))
def test_fixture_structure(layout, n):
    meta, idx, val = read(layout, n)
    assert len(idx) == 4096 and np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < n ** 3
    assert meta["tol10_rel_res"] <= 1e-10 and meta["tol12_rel_res"] <= 1e-12
    assert meta["tol12_cycles"] > meta["tol10_cycles"] > 5
    # the two stopping points differ by about the 1e-10 residual, far below the solution
    rms12 = meta["tol12_norm2"] / np.sqrt(float(n) ** 3)
    d = val[:, 0] - val[:, 1]
    assert np.sqrt(np.mean(d ** 2)) < 1e-8 * rms12
    assert abs(meta["tol12_mean"]) < 1e-12 * rms12


def test_drop_film128_fixture_is_current():
    meta, idx, val = read("drop_film", 128)
    wl = W.drop_film_workload(128)
    beta = oracle.faces_from_vof(wl.f_drop, wl.f_film, wl.rho_drop, wl.rho_film, wl.rho_gas)
    b = oracle.divergence(wl.u, wl.v, wl.w, wl.h, wl.dt)
    for col, (name, tol) in enumerate((("tol10", 1e-10), ("tol12", 1e-12))):
        res = oracle.solve(beta, b, wl.h, tol=tol, max_cycles=60)
        assert res.cycles == meta[f"{name}_cycles"]
        np.testing.assert_allclose(res.p.ravel()[idx], val[:, col], rtol=1e-12, atol=1e-14)
