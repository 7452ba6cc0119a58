"""GPU parity for the half-integer Matern kernels (Sec. 3.1): the closed-form
factor kernel against the oracle's quadrature, dense Gram blocks, and a
solve + posterior against the dense Cholesky oracle."""
import dataclasses

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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("code", [2, 3, 4])          # Matern 3/2, 5/2, 7/2
@pytest.mark.parametrize("ell", [0.1, 0.3])
def test_matern_factor_kernel_matches_quadrature(G, code, ell):
    q = code - 1
    rng = np.random.default_rng(9)
    e1 = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, 11)]))
    e2 = np.linspace(0.0, 1.0, 30)
    x = rng.uniform(-0.1, 1.1, 9)
    for p in range(q + 1):
        for qq in range(q + 1):
            for kind, a1, a2, ref in [
                (0, e1, e2, O.cell_cell(p, qq, e1, e2, ell, kq=q)),
                (1, x, e2, O.point_cell(p, qq, x, e2, ell, kq=q)),
                (2, x, e1, O.point_point(p, qq, x, e1, ell, kq=q)),
            ]:
                out = torch.empty(ref.size, dtype=torch.float64, device="cuda:0")
                G.factor(kind, p, qq, a1, a2, ell, out, kernel=code)
                got = host(out).reshape(ref.shape)
                scale = np.abs(ref).max()
                assert np.abs(got - ref).max() <= 1e-11 * scale, (kind, p, qq, np.abs(got - ref).max() / scale)


def _matern(p, codes):
    return dataclasses.replace(p, kernel=codes, name=p.name + "_matern")


SMALL = {
    "heat1d_m32_m52": lambda: _matern(W.heat1d_c1(), (2, 3)),
    "advdiff_6x7_m52": lambda: _matern(W.advdiff_c2(nt=6, nx=7, n_ic=10), (3, 3)),
    "wave_3x4x5_m52": lambda: _matern(W.wave2d_c4(nt=3, nx=4, ny=5, n_ic=4, n_bt=3, n_bs=2), (3, 3, 3)),
    "heat2d_3x4x3_m72": lambda: _matern(W.heat2d_c3(nt=3, nx=4, ny=3, n_ic=4, n_bt=3, n_bs=2), (4, 4, 4)),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_matern_dense_gram_matches_oracle(G, name):
    p = SMALL[name]()
    ref = O.Oracle(p).gram()
    h = G.assemble(p, max_iter=8)
    try:
        n = ref.shape[0]
        out = torch.empty(n * n, dtype=torch.float64, device="cuda:0")
        G.gram_block(h, 0, n, 0, n, out)
        got = host(out).reshape(n, n)
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
        x = np.random.default_rng(4).standard_normal(n)
        y = torch.empty(n, dtype=torch.float64, device="cuda:0")
        G.matvec(h, torch.as_tensor(x, device="cuda:0"), y)
        assert relerr(host(y), ref @ x) <= 1e-11
    finally:
        G.destroy(h)


def test_matern_heat1d_posterior_matches_cholesky(G):
    p = SMALL["heat1d_m32_m52"]()
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    m_ref, v_ref, _ = O.dense_posterior(o, X)
    h = G.assemble(p, max_iter=256)
    try:
        info = G.solve(h, tol=1e-10, max_iter=256, check_every=4)
        assert info["rel_res"] <= 1e-8, info
        M = len(X)
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean, var)
        assert_close(host(mean), m_ref, 1e-6, converged=True)
        assert np.all(host(var) >= v_ref - 1e-9)
    finally:
        G.destroy(h)
