"""GPU parity of the coarse-scheme warm start (appendix "Multigrid
preconditioners") through the C-ABI: the coarse block (exact conditioning on
nested coarse volumes) followed by k CG iterations, against the float64
oracle's itergp_coarse; convergence on advection-diffusion 128^2 against the
plain solve; and the option checks."""
import time

import numpy as np
import pytest

import workloads as W
from parity import assert_close
from oracle import gpfvm_oracle as O
from oracle.gpfvm_oracle import SchurSystem, two_stage_posterior

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_05020_amd as G
    G.lib()
    return G


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


CASES = {
    "heat1d_16x16": (lambda: W.heat1d_c1(), [(4, 4), (2, 2)]),
    "advdiff_12x10": (lambda: W.advdiff_c2(nt=12, nx=10, n_ic=20), [(3, 5), (2, 2)]),
    "wave_4x6x5": (lambda: W.wave2d_c4(nt=4, nx=6, ny=5, n_ic=6, n_bt=3, n_bs=3, grid_t=3), [(2, 3, 5), (2, 2, 1)]),
}
RUNS = [(c, f, k) for c, (_, fs) in CASES.items() for f in fs for k in (0, 5, 20)]


def _posterior(G, h, p):
    M = int(np.prod([len(a) for a in p.grid]))
    mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
    var = torch.empty(M, dtype=torch.float64, device="cuda:0")
    G.posterior(h, p.grid, mean, var)
    return host(mean), host(var)


@pytest.mark.parametrize("case,f,k", RUNS)
def test_coarse_warm_start_matches_oracle(G, case, f, k):
    p = CASES[case][0]()
    o = O.Oracle(p)
    S = SchurSystem(o)
    Cm = O.coarse_aggregation(p, f)
    nc = Cm.shape[0]
    v, D, eta, _ = O.itergp_coarse(S, Cm, k, passes=2)
    X = o.grid_points(p.grid)
    m_ref, v_ref = two_stage_posterior(S, v, X, D, eta)
    h = G.assemble(p, max_iter=nc + k + 1)
    try:
        info = G.solve(h, tol=0.0, max_iter=k, check_every=4, reorth_passes=2, coarsen=f)
        assert info["rc"] == G.OK and info["coarse"] == nc and info["iters"] == nc + k, info
        m, var = _posterior(G, h, p)
    finally:
        G.destroy(h)
    assert_close(m, m_ref, 1e-6)
    assert_close(var, v_ref, 1e-6)


# The 4 x 4 coarse block (1024 coarse cells, coarse Gram of condition ~1e9) leaves
# the CG phase an attainable relative residual of about 1e-8 (measured minimum
# 9e-9 after 24 iterations); the stopping tolerance of the comparison sits above it.
COARSE_TOL = 3e-8


def test_coarse_warm_start_converges_with_fewer_cg_iterations(G):
    """advection-diffusion 128 x 128 cells to 3e-8: the same posterior mean as
    the plain solve, with fewer CG iterations after the coarse block."""
    p = W.advdiff_c2()
    M = int(np.prod([len(a) for a in p.grid]))
    res = {}
    for f in (None, (8, 8), (4, 4)):
        h = G.assemble(p, max_iter=2048)
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = G.solve(h, tol=COARSE_TOL, max_iter=1024, coarsen=f)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
            G.posterior(h, p.grid, mean)
            res[f] = (info, host(mean), dt)
        finally:
            G.destroy(h)
        i = res[f][0]
        print(f"coarsen={f}: {i['coarse']} coarse + {i['iters'] - i['coarse']} CG directions, "
              f"rel_res {i['rel_res']:.2e}, solve {1e3 * dt:.2f} ms", flush=True)
    plain = res[None]
    assert plain[0]["rc"] == G.OK
    for f in ((8, 8), (4, 4)):
        info, m, _ = res[f]
        assert info["rc"] == G.OK and info["rel_res"] <= COARSE_TOL, info
        assert info["iters"] - info["coarse"] < plain[0]["iters"], (info, plain[0])
        assert_close(m, plain[1], 1e-6, converged=True)


def test_tolerance_below_attainable_accuracy_rolls_back(G):
    """A stopping tolerance below the attainable accuracy (1e-10 with the 4 x 4
    coarse block) stalls the recursive residual; the iterations after that lose
    conjugacy and the residual grows without bound.  The solve stops once it has
    grown 1000-fold above its smallest value and returns the state at that
    smallest value: NOCONV, a residual near the attainable 1e-8, a handful of
    directions past the coarse block, and a posterior mean equal to the one
    converged to COARSE_TOL."""
    p = W.advdiff_c2()
    M = int(np.prod([len(a) for a in p.grid]))
    out = {}
    for tol in (COARSE_TOL, 1e-10):
        h = G.assemble(p, max_iter=2048)
        try:
            info = G.solve(h, tol=tol, max_iter=1024, coarsen=(4, 4))
            err = G.last_error(h)
            mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
            G.posterior(h, p.grid, mean)
            out[tol] = (info, err, host(mean))
        finally:
            G.destroy(h)
    info, err, m = out[1e-10]
    ref_info, _, ref = out[COARSE_TOL]
    assert ref_info["rc"] == G.OK
    assert info["rc"] == G.E_NOCONV and "rolled back" in err, (info, err)
    assert info["rel_res"] <= COARSE_TOL, info
    assert info["iters"] - info["coarse"] <= 64, info
    assert np.all(np.isfinite(m))
    assert_close(m, ref, 1e-6, converged=True)


def test_coarse_option_checks(G):
    p = W.heat1d_c1()
    h = G.assemble(p, max_iter=32)
    try:
        for kw in [dict(coarsen=(3, 4)),                       # 3 does not divide 16
                   dict(coarsen=(0, 1)),
                   dict(coarsen=(2, 2)),                       # 64 coarse cells >= max_iter 32
                   dict(coarsen=(4, 4), prec=G.PREC_MIXED),
                   dict(coarsen=(4, 4), reorth_passes=1)]:
            with pytest.raises(G.GpfvmError) as e:
                G.solve(h, tol=0.0, max_iter=4, **kw)
            assert e.value.code == G.E_INVALID, kw
        info = G.solve(h, tol=0.0, max_iter=4, coarsen=(4, 4))
        assert info["coarse"] == 16 and info["iters"] == 20
        with pytest.raises(G.GpfvmError) as e:                  # no warm start on resume
            G.solve(h, tol=0.0, max_iter=4, resume=True, coarsen=(4, 4))
        assert e.value.code == G.E_INVALID
        info = G.solve(h, tol=0.0, max_iter=4, resume=True)      # plain resume continues
        assert info["iters"] == 24
    finally:
        G.destroy(h)
