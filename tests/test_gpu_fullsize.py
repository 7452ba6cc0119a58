"""GPU parity at the full advection-diffusion size (128 x 128 volumes + 256
initial points, the configuration bench.py times): the volume-system operator
element by element, and the solve + posterior on sampled grid points against
the oracle's IterGP with the same recurrences."""
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


@pytest.fixture(scope="module")
def c2():
    p = W.advdiff_c2()
    o = O.Oracle(p)
    return p, o, SchurSystem(o)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def test_schur_operator_matches_oracle(G, c2):
    """nrhs = 1 applies the point correction Q^T Q (Q = L^{-1} G_bp) in
    factored form, the initial points being one group pinned at t = 0;
    nrhs = 2 through the cross-block Kronecker products and the point-block
    triangular solves.  Both against the oracle's Cholesky."""
    p, o, S = c2
    rng = np.random.default_rng(5)
    X = rng.standard_normal((2, p.n_pde))
    h = G.assemble(p, max_iter=8)
    try:
        x1 = torch.as_tensor(X[0], device="cuda:0")
        y1 = torch.empty_like(x1)
        G.schur_matvec(h, x1, y1, nrhs=1)
        assert relerr(host(y1), S.matvec(X[0])) <= 1e-11
        x = torch.as_tensor(X.ravel(), device="cuda:0")
        y = torch.empty_like(x)
        G.schur_matvec(h, x, y, nrhs=2)
        Y = host(y).reshape(2, -1)
        for r in range(2):
            assert relerr(Y[r], S.matvec(X[r])) <= 1e-11
        y32 = torch.empty_like(x)
        G.schur_matvec(h, x, y32, nrhs=2, prec=G.PREC_MIXED)
        e = relerr(host(y32), host(y))
        assert e <= 1e-5, e
    finally:
        G.destroy(h)


def _sample(p, k=384, seed=1):
    X = O.Oracle(p).grid_points(p.grid)
    idx = np.random.default_rng(seed).choice(len(X), size=k, replace=False)
    return X, idx


def test_converged_solve_matches_oracle_itergp(G, c2):
    p, o, S = c2
    X, idx = _sample(p)
    vp, D, eta, res = O.itergp(S, 2000, tol=1e-8, passes=2)
    m_ref, _ = two_stage_posterior(S, vp, X[idx])
    h = G.assemble(p, max_iter=2048)
    try:
        info = G.solve(h, tol=1e-8, max_iter=2048, check_every=16)
        assert info["rc"] == G.OK, info
        assert info["rel_res"] <= 1e-8, info
        assert abs(info["iters"] - D.shape[1]) <= 3, (info["iters"], D.shape[1])
        M = len(X)
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean, var)
        m = host(mean)
        assert_close(m[idx], m_ref, 1e-6, converged=True)
        v = host(var)
        assert np.all(np.isfinite(v)) and v.min() > -1e-9 and v.max() <= 1.0 + 1e-12
    finally:
        G.destroy(h)


def test_fixed_iteration_posterior_matches_oracle(G, c2):
    """Early-terminated IterGP (120 iterations): mean and combined variance."""
    p, o, S = c2
    X, idx = _sample(p, seed=2)
    k = 120
    vp, D, eta, _ = O.itergp(S, k, passes=2)
    m_ref, v_ref = two_stage_posterior(S, vp, X[idx], D, eta)
    h = G.assemble(p, max_iter=k)
    try:
        info = G.solve(h, tol=0.0, max_iter=k, check_every=16)
        assert info["iters"] == k
        M = len(X)
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean, var)
        assert_close(host(mean)[idx], m_ref, 1e-6)
        assert_close(host(var)[idx], v_ref, 1e-6)
    finally:
        G.destroy(h)


@pytest.mark.parametrize("name,B,checked", [("wave2d_64x128x128", 1, [0]), ("heat2d_64x64x64", 64, [0, 31, 63])])
def test_full_size_volume_matvec_matches_oracle(G, name, B, checked):
    """The volume Gram (plus noise) at full size, in the launch configuration of
    bench.py's extra rooflines (wave 64x128x128 with 1 rhs; heat 64^3 with 64
    rhs), compared on whole right-hand sides with the oracle's Kronecker
    matvec over the quadrature factors."""
    p = {"wave2d_64x128x128": W.wave2d_c4, "heat2d_64x64x64": W.heat2d_c3}[name]()
    assert p.name == name
    o = O.Oracle(p)
    rng = np.random.default_rng(21)
    X = rng.standard_normal((B, p.n_pde))
    h = G.assemble(p, max_iter=8)
    try:
        x = torch.as_tensor(X.ravel(), device="cuda:0")
        y = torch.empty_like(x)
        G.volume_matvec(h, x, y, nrhs=B)
        Y = host(y).reshape(B, -1)
    finally:
        G.destroy(h)
    noise = o.noise_pde()
    for r in checked:
        ref = o.volume_matvec(X[r]) + noise * X[r]
        assert relerr(Y[r], ref) <= 1e-11, (r, relerr(Y[r], ref))
