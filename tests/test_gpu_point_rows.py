"""The one-right-hand-side point-block solve by row-streaming triangular
products (Sec. 4.2: the point block is conditioned exactly through its
Cholesky factor).  A 3-D problem whose point block is too large for the
one-workgroup solve (n_b > 512) and whose correction Q = L^{-1} G_bp is too
large to stay resident (8 n_b N > 256 MiB) takes this path on every operator
application of the solver loop, as the large 3-D workloads and most serving
requests do.  Compared with the oracle's LAPACK Cholesky: the operator
element by element, an early-terminated IterGP posterior through the
single-handle entry points, and the same request served by the
continuous-batching server."""
import numpy as np
import pytest

import workloads as W
from parity import assert_close
from oracle import gpfvm_oracle as O
from oracle.gpfvm_oracle import SchurSystem, two_stage_posterior

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

K_ITERS = 12


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_05020_amd as G
    G.lib()
    return G


@pytest.fixture(scope="module")
def case():
    # 24 x 32 x 32 volumes, 32^2 initial + 4 x 24 x 16 boundary points: n_b = 2560
    p = W.heat2d_request(32, 24, seed=4242)
    assert p.n_b > 512 and 8 * p.n_b * p.n_pde > (256 << 20)
    o = O.Oracle(p)
    S = SchurSystem(o)
    X = o.grid_points(p.grid)
    idx = np.sort(np.random.default_rng(3).choice(len(X), size=256, replace=False))
    vp, D, eta, _ = O.itergp(S, K_ITERS, passes=2)
    m_ref, v_ref = two_stage_posterior(S, vp, X[idx], D, eta)
    return p, S, idx, m_ref, v_ref


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_operator_through_row_streaming_solves(G, case):
    p, S, _, _, _ = case
    rng = np.random.default_rng(31)
    h = G.assemble(p, max_iter=8)
    try:
        for rep in range(2):
            x = rng.standard_normal(p.n_pde)
            y = torch.empty(p.n_pde, dtype=torch.float64, device="cuda:0")
            G.schur_matvec(h, torch.as_tensor(x, device="cuda:0"), y, nrhs=1)
            ref = S.matvec(x)
            got = host(y)
            e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            assert e <= 1e-10, (rep, e)
            assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref)), rep
    finally:
        G.destroy(h)


def test_early_terminated_posterior(G, case):
    p, _, idx, m_ref, v_ref = case
    h = G.assemble(p, max_iter=K_ITERS)
    try:
        info = G.solve(h, tol=0.0, max_iter=K_ITERS, check_every=4)
        assert info["iters"] == K_ITERS, info
        M = int(np.prod([len(a) for a in p.grid]))
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean, var)
        assert_close(host(mean)[idx], m_ref, 1e-6, what="mean")
        assert_close(host(var)[idx], v_ref, 1e-6, what="var")
    finally:
        G.destroy(h)


def test_served_request_matches_oracle(G, case):
    p, _, idx, m_ref, v_ref = case
    with G.Server(workers=2, hbm_budget=32 << 30, prec=G.PREC_FP64, tol=0.0, max_iter=K_ITERS) as srv:
        other = srv.submit(W.heat2d_request(16, 16, seed=4243))     # a second request in flight
        done, res, m, v = srv.poll(srv.submit(p), wait=True)
        srv.poll(other, wait=True)
    assert done and res["rc"] == G.OK and res["iters"] == K_ITERS, res
    assert_close(m[idx], m_ref, 1e-6, what="served mean")
    assert_close(v[idx], v_ref, 1e-6, what="served var")
