"""The 2-D wave benchmark (appendix "2D Wave Equation Benchmark") as a pin of
the Matérn-5/2 oracle: its exact solution follows from separation of
variables, so the oracle's posterior mean must approach it as the FVM scheme
refines, independently of any GP-FVM arithmetic."""
import numpy as np

import workloads as W
from oracle import gpfvm_oracle as O


def test_exact_solution_satisfies_the_ibvp():
    """The closed form solves u_tt = u_xx + u_yy (second differences), and the
    benchmark's IC/BC data are its values (u, u_t at t = 0, 0 on the edges)."""
    seed = 3
    h = 1e-3
    t0, x0, y0 = np.array([0.37, 1.21]), np.array([0.23, 0.61]), np.array([0.44, 0.8])

    def u(t, x, y):
        return W.wave2d_benchmark_solution(seed, [t, x, y]).reshape(len(t), len(x), len(y))

    utt = (u(t0 + h, x0, y0) - 2 * u(t0, x0, y0) + u(t0 - h, x0, y0)) / h ** 2
    uxx = (u(t0, x0 + h, y0) - 2 * u(t0, x0, y0) + u(t0, x0 - h, y0)) / h ** 2
    uyy = (u(t0, x0, y0 + h) - 2 * u(t0, x0, y0) + u(t0, x0, y0 - h)) / h ** 2
    assert np.max(np.abs(utt - uxx - uyy)) <= 1e-4 * np.max(np.abs(utt))
    p = W.wave2d_benchmark(n=4, seed=seed)
    g_u, g_ut = p.groups[0], p.groups[1]
    assert np.allclose(g_u.y, W.wave2d_benchmark_solution(seed, g_u.axes), atol=1e-14)
    ut = (W.wave2d_benchmark_solution(seed, [np.array([h])] + g_ut.axes[1:])
          - W.wave2d_benchmark_solution(seed, [np.array([-h])] + g_ut.axes[1:])) / (2 * h)
    assert np.max(np.abs(ut)) <= 1e-12 and np.all(g_ut.y == 0)
    for g in p.groups[2:]:
        assert np.max(np.abs(W.wave2d_benchmark_solution(seed, g.axes))) <= 1e-14 and np.all(g.y == 0)
    assert p.n_b == 64 + 64 + 4 * 20 * 10


def test_matern_posterior_converges_to_the_exact_solution():
    """Relative L2 error of the exact posterior mean on an 8 x 16 x 16 grid
    falls as the scheme refines (n^3 volumes), and is below 15% at n = 16."""
    errs = []
    for n in (8, 12, 16):
        p = W.wave2d_benchmark(n=n)
        o = O.Oracle(p)
        X = o.grid_points(p.grid)
        m, v, _ = O.dense_posterior(o, X)
        u = W.wave2d_benchmark_solution(0, p.grid)
        errs.append(np.linalg.norm(m - u) / np.linalg.norm(u))
        assert np.all(v >= -1e-9)
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.15, errs

