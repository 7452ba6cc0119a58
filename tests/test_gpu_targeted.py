"""GPU parity of targeted uncertainty reduction (appendix "Targeted
uncertainty reduction") through the C-ABI against the float64 oracle: a
solve of k IterGP iterations, then m iterations whose actions are the
residuals of K_S(X~) beta_i, the weights beta_i drawn on the host (Dirichlet)
and passed to both sides.  Posterior mean and combined variance afterwards
within 1e-6 relative (the float64 target), plus the error paths."""
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


def _target_axes(p, frac):
    """A tensor sub-grid of the evaluation grid: the last `frac` of time and
    the middle of every spatial axis (the region whose uncertainty is
    targeted)."""
    axes = []
    for i, a in enumerate(p.grid):
        n = len(a)
        if i == 0:
            axes.append(np.asarray(a[int(n * (1 - frac)):], dtype=np.float64))
        else:
            axes.append(np.asarray(a[n // 4: n - n // 4], dtype=np.float64))
    return axes


CASES = {
    "heat1d_16x16": lambda: W.heat1d_c1(),
    "advdiff_12x10": lambda: W.advdiff_c2(nt=12, nx=10, n_ic=20),
    "wave_4x6x5": lambda: W.wave2d_c4(nt=4, nx=6, ny=5, n_ic=6, n_bt=3, n_bs=3, grid_t=3),
}


# (case, k solve iterations, m targeted iterations): m kept where the last eta
# stays above ~1e-9 of the first (beyond that the directions are rounding noise)
RUNS = [(c, k, m) for c in CASES for (k, m) in [(0, 3), (5, 6), (12, 10 if c.startswith("heat1d") else 30)]]


@pytest.mark.parametrize("case,k,m", RUNS)
def test_targeted_refinement_matches_oracle(G, case, k, m):
    p = CASES[case]()
    o = O.Oracle(p)
    S = SchurSystem(o)
    Xe = o.grid_points(p.grid)
    axes = _target_axes(p, 0.5)
    Xt = o.grid_points(axes)
    rng = np.random.default_rng(11 + k + m)
    betas = rng.dirichlet(np.ones(Xt.shape[0]), size=m)
    # oracle
    vp, D, eta, _ = O.itergp(S, k, passes=2)
    KS = O.schur_cross(S, Xt)
    v2, D2, e2, _ = O.itergp_targeted(S, vp, D, eta, KS, betas, passes=2)
    assert D2.shape[1] == k + m
    m_ref, var_ref = two_stage_posterior(S, v2, Xe, D2, e2)
    # GPU
    h = G.assemble(p, max_iter=k + m)
    try:
        info = G.solve(h, tol=0.0, max_iter=k, check_every=4, reorth_passes=2)
        assert info["iters"] == k
        M = Xe.shape[0]
        mean0 = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var0 = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean0, var0)
        var_before = host(var0)
        r = G.refine_variance(h, axes, betas)
        assert r["rc"] == G.OK and r["iters"] == k + m, r
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean, var)
        got_m, got_v = host(mean), host(var)
    finally:
        G.destroy(h)
    assert_close(got_m, m_ref, 1e-6)
    assert_close(got_v, var_ref, 1e-6)
    # more directions never raise the combined variance
    assert np.all(got_v <= var_before + 1e-9 * np.max(np.abs(var_before)))


def test_targeted_refinement_error_paths(G):
    p = W.heat1d_c1()
    axes = _target_axes(p, 0.5)
    Mt = int(np.prod([len(a) for a in axes]))
    w = np.full((2, Mt), 1.0 / Mt)
    h = G.assemble(p, max_iter=6)
    try:
        with pytest.raises(G.GpfvmError) as e:           # before any solve
            G.refine_variance(h, axes, w)
        assert e.value.code == G.E_STATE
        G.solve(h, tol=0.0, max_iter=5, reorth_passes=2)
        with pytest.raises(G.GpfvmError) as e:           # 5 + 2 directions > max_iter 6
            G.refine_variance(h, axes, w)
        assert e.value.code == G.E_INVALID
        with pytest.raises(ValueError):                  # weights of the wrong width
            G.refine_variance(h, axes, np.ones((1, Mt + 1)))
        bad = w[:1].copy()
        bad[0, 0] = np.nan
        with pytest.raises(G.GpfvmError) as e:
            G.refine_variance(h, axes, bad)
        assert e.value.code == G.E_INVALID
        r = G.refine_variance(h, axes, w[:1])            # one more fits
        assert r["rc"] == G.OK and r["iters"] == 6
        G.solve(h, tol=0.0, max_iter=4, reorth_passes=1)  # one-pass solve: no S D images
        with pytest.raises(G.GpfvmError) as e:
            G.refine_variance(h, axes, w[:1])
        assert e.value.code == G.E_STATE
    finally:
        G.destroy(h)
