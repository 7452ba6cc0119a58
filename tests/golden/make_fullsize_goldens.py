"""Write the stored oracle values for the full-size 3-D problems: the wave
problem (64 x 128 x 128 volumes with per-cell c^2, 16384 initial/boundary
points; default); with the argument heat2d, the 2-D heat problem
(64 x 64 x 64 volumes, 12288 initial/boundary points); with the argument
shallow_water, the linearised shallow-water system at the paper's tsunami
scale (20 x 90 x 170 cells, three equations and three outputs: 918 000 volume
observations; 18 380 initial and radiation-boundary points).

Calls only the oracle: the two-stage system (exact Cholesky conditioning on
the points, Sec. 4.2) and IterGP with CG actions and the projection done twice
(Sec. 4.1; the Limitations section's full reorthogonalisation), stopped early
after a fixed number of iterations.  The posterior mean and the combined
variance (Sec. 2.1 eq. lin-cond-mean / lin-cond-cov with the IterGP inverse
approximation) are stored at 256 seeded sample points of the 8 x 128 x 128
evaluation grid of cell centres, after 30 and after 200 iterations (the
second run continues the first, with the same recurrences).  For the heat
problem: after 30 iterations, at 256 points of its 16 x 64 x 64 grid.  For
the shallow-water system: after 20 iterations, every output (h, u, v) at 128
points of its 4 x 90 x 170 grid.

Run from the repository root:  python tests/golden/make_fullsize_goldens.py [heat2d]
(wave: about half an hour on 8 cores, writes tests/golden/wave2d_c4_itergp.json;
heat2d: a few minutes, writes tests/golden/heat2d_c3_itergp.json;
shallow_water: about half an hour, writes tests/golden/shallow_water_itergp.json).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W                                     # noqa: E402
from oracle import gpfvm_oracle as O                      # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = {
    "wave2d": (W.wave2d_c4, os.path.join(HERE, "wave2d_c4_itergp.json"), (30, 200), 4, 256),
    "heat2d": (W.heat2d_c3, os.path.join(HERE, "heat2d_c3_itergp.json"), (30,), 3, 256),
    "shallow_water": (W.shallow_water, os.path.join(HERE, "shallow_water_itergp.json"), (20,), 6, 128),
}


def main(case="wave2d"):
    make, OUT, STOPS, SAMPLE_SEED, N_SAMPLE = CASES[case]
    t0 = time.perf_counter()
    p = make()
    o = O.Oracle(p)
    S = O.SchurSystem(o)
    X = o.grid_points(p.grid)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(len(X), size=N_SAMPLE, replace=False))
    print(f"setup {time.perf_counter() - t0:.0f}s", flush=True)
    out = {"workload": p.name, "n_pde": int(p.n_pde), "n_b": int(p.n_b),
           "grid": [len(a) for a in p.grid], "passes": 2, "sample_seed": SAMPLE_SEED,
           "idx": idx.tolist(), "stops": {}}
    state = None
    done = 0
    for k in STOPS:
        vp, D, eta, res = O.itergp(S, k - done, passes=2, init=state)
        state = (vp, D, eta)
        done = k
        assert D.shape[1] == k, (D.shape, k)
        rr = float(np.linalg.norm(S.b - S.matvec(vp)) / np.linalg.norm(S.b))
        if p.nout == 1:
            m, v = O.two_stage_posterior(S, vp, X[idx], D, eta)
            out["stops"][str(k)] = {"mean": [float(x) for x in m], "var": [float(x) for x in v], "rel_res": rr}
        else:                       # one list per output
            mv = [O.two_stage_posterior(S, vp, X[idx], D, eta, out=j) for j in range(p.nout)]
            out["stops"][str(k)] = {"mean": [[float(x) for x in m] for m, _ in mv],
                                    "var": [[float(x) for x in v] for _, v in mv], "rel_res": rr}
        print(f"k={k}: rel_res {rr:.3e}, {time.perf_counter() - t0:.0f}s", flush=True)
        with open(OUT + ".tmp", "w") as f:
            json.dump(out, f)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "wave2d")
