"""The full-size wave problem (64 x 128 x 128 volumes with per-cell c^2,
16384 initial/boundary points) in the configuration bench.py times: assemble,
early-terminated IterGP with CG actions (Sec. 4.1), posterior mean and
combined variance on the 8 x 128 x 128 grid (Sec. 2.1, Sec. 4.1-4.2).
Compared at 256 sampled grid points with the oracle's values after the same
numbers of iterations, stored under tests/golden by a script that calls only
the oracle (tests/golden/make_wave_c4_golden.py)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from parity import assert_close

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "wave2d_c4_itergp.json")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_05020_amd as G
    G.lib()
    return G


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("k", [30, 200])
def test_wave_fullsize_itergp_posterior_matches_oracle(G, golden, k):
    ref = golden["stops"][str(k)]
    p = W.wave2d_c4()
    assert p.name == golden["workload"] and p.n_b == golden["n_b"]
    idx = np.asarray(golden["idx"])
    h = G.assemble(p, max_iter=k)
    try:
        print(f"wave 64x128x128, {k} IterGP iterations", flush=True)
        info = G.solve(h, tol=0.0, max_iter=k, check_every=50)
        assert info["iters"] == k, info
        M = int(np.prod([len(a) for a in p.grid]))
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean, var)
        torch.cuda.synchronize()
        m, v = mean.cpu().numpy(), var.cpu().numpy()
    finally:
        G.destroy(h)
    assert abs(info["rel_res"] - ref["rel_res"]) <= 1e-6 * ref["rel_res"] + 1e-12, (info["rel_res"], ref["rel_res"])
    assert_close(m[idx], ref["mean"], 1e-6, what="mean")
    assert_close(v[idx], ref["var"], 1e-6, what="var")
    # the whole grid: finite, and the combined variance stays within [0, sf2]
    assert np.all(np.isfinite(m)) and np.all(np.isfinite(v))
    assert v.min() >= -1e-9 and v.max() <= 1.0 + 1e-12
