"""Writes tests/golden/<layout><N>_oracle.txt: sampled values of the oracle's
solutions of one seeded workload, FP64 V-cycles (2+2 red-black sweeps) from a
zero guess, stopped at two relative residuals:
  tol10  ||r|| <= 1e-10 ||b||  (the stopping rule of the benchmark solve)
  tol12  ||r|| <= 1e-12 ||b||  (converged: reference for a tighter GPU solve)
Calls only the oracle and the seeded input generator.

Run: python tests/golden/make_oracle_samples.py many_drops 512     (about 10 GB of host memory, minutes)
     python tests/golden/make_oracle_samples.py drop_film 128
     python tests/golden/make_oracle_samples.py spheroid_film 256
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_30082_amd import workloads as W  # noqa: E402

NSAMPLES = 4096
SAMPLE_SEED = 4
TOLS = (("tol10", 1e-10), ("tol12", 1e-12))


LAYOUT_TEXT = {
    "many_drops": "film + 32 drops workload (seeded inputs: velocity 0,\n# drops 1)",
    "drop_film": "film + one drop workload (seeded input: velocity 0)",
    "spheroid_film": "film + oblate spheroid workload (seeded input: velocity 0)",
    "sphere": "sphere workload (seeded input: velocity 0)",
}


def main():
    layout, N = sys.argv[1], int(sys.argv[2])
    t0 = time.time()
    wl = W.make(layout, N)
    beta = oracle.faces_from_vof(wl.f_drop, wl.f_film, wl.rho_drop, wl.rho_film, wl.rho_gas)
    b = oracle.divergence(wl.u, wl.v, wl.w, wl.h, wl.dt)
    del wl
    print(f"inputs {time.time() - t0:.1f} s", flush=True)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(N ** 3, NSAMPLES, replace=False))
    cols, meta = [], []
    for name, tol in TOLS:
        res = oracle.solve(beta, b, 1.0 / N, tol=tol, max_cycles=60)
        print(f"{name} {time.time() - t0:.1f} s: {res.cycles} cycles, rr {res.rel_res:.3e}", flush=True)
        p = res.p.ravel()
        cols.append(p[idx].copy())
        meta.append((name, res.cycles, res.rel_res, float(np.linalg.norm(p)), float(p.mean()),
                     res.rhs_mean))
        del res, p
    out = os.path.join(HERE, f"{layout}{N}_oracle.txt")
    with open(out, "w") as f:
        f.write(f"# Oracle solutions of the {N}^3 {LAYOUT_TEXT[layout]}, FP64 V-cycles (2+2 red-black\n")
        f.write("# sweeps) from a zero guess, stopped at ||r|| <= 1e-10 ||b|| (tol10) and\n")
        f.write("# ||r|| <= 1e-12 ||b|| (tol12).\n")
        f.write(f"# Written by tests/golden/make_oracle_samples.py {layout} {N}, which calls only oracle/.\n")
        for name, cyc, rr, n2, mean, rm in meta:
            f.write(f"# {name}_cycles {cyc}\n# {name}_rel_res {rr:.17g}\n")
            f.write(f"# {name}_norm2 {n2:.17g}\n# {name}_mean {mean:.17g}\n")
        f.write(f"# rhs_mean {meta[0][5]:.17g}\n# sample_seed {SAMPLE_SEED}\n")
        f.write("# flat_index value_tol10 value_tol12\n")
        for k, i in enumerate(idx):
            f.write(f"{int(i)} {cols[0][k]:.17g} {cols[1][k]:.17g}\n")
    print(f"wrote {out} in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
