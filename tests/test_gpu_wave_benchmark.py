"""The 2-D wave benchmark (appendix "2D Wave Equation Benchmark") on the HIP
path: Matérn-5/2 in every dimension, u and u_t observed at t = 0, Dirichlet
edges.  At n = 12 the posterior mean equals the oracle's exact (Cholesky)
posterior to 1e-6; at n = 16, 24, 32 (32^3 = 8^5 volumes, the largest scheme
of the paper's figure) the error against the separation-of-variables solution
falls below 2%."""
import numpy as np
import pytest

import workloads as W
from parity import assert_close
from oracle import gpfvm_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_05020_amd as G
    G.lib()
    return G


def _gpu_posterior(G, p, tol):
    h = G.assemble(p, max_iter=min(p.n_pde, 4000))
    try:
        info = G.solve(h, tol=tol, max_iter=min(p.n_pde, 4000), check_every=16)
        M = int(np.prod([len(a) for a in p.grid]))
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean, var)
        torch.cuda.synchronize()
        return mean.cpu().numpy(), var.cpu().numpy(), info
    finally:
        G.destroy(h)


def test_wave_benchmark_matches_cholesky_oracle(G):
    p = W.wave2d_benchmark(n=12)
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    m_ref, v_ref, _ = O.dense_posterior(o, X)
    m, v, info = _gpu_posterior(G, p, 1e-10)
    assert info["rc"] == G.OK and info["rel_res"] <= 1e-10, info
    assert_close(m, m_ref, 1e-6, converged=True)
    assert np.all(v >= v_ref - 1e-9)                 # combined >= exact variance


def test_wave_benchmark_converges_to_the_exact_solution(G):
    errs = []
    for n in (16, 24, 32):
        p = W.wave2d_benchmark(n=n)
        m, v, info = _gpu_posterior(G, p, 1e-8)
        assert info["rc"] == G.OK, (n, info)
        u = W.wave2d_benchmark_solution(0, p.grid)
        errs.append(np.linalg.norm(m - u) / np.linalg.norm(u))
        print(f"wave benchmark n={n}: {info['iters']} iterations, relative error {errs[-1]:.3e}", flush=True)
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[0] < 0.15 and errs[1] < 0.05 and errs[2] < 0.02, errs
