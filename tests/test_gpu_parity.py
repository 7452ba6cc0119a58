"""GPU parity: the HIP path (through the C-ABI) against the float64 CPU oracle.

Tolerances (float64 path): factors and Gram entries are closed forms whose
only error is rounding, amplified by the second-difference cancellation of
the antiderivative form by about (lengthscale / cell width)^2 (< 300 here), so
1e-11 of the matrix scale; matvecs sum <= 10^3 terms of those, 1e-11 relative.
Posterior mean and variance: 1e-6 relative (the float64 target)."""
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


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# ---------------------------------------------------------------------------
# 1-D factors
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pq", [(0, 0), (1, 0), (0, 1), (1, 1), (2, 0), (0, 2), (2, 2), (4, 0), (1, 3), (0, 4)])
@pytest.mark.parametrize("ell", [0.1, 0.3])
def test_factor_kernel_matches_quadrature(G, pq, ell):
    p, q = pq
    rng = np.random.default_rng(7)
    e1 = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, 11)]))    # 12 ragged cells
    e2 = np.linspace(0.0, 1.0, 38)                                        # 37 uniform cells
    x = rng.uniform(-0.1, 1.1, 9)
    for kind, a1, a2, ref in [
        (0, e1, e2, O.cell_cell(p, q, e1, e2, ell)),
        (1, x, e2, O.point_cell(p, q, x, e2, ell)),
        (2, x, e1, O.point_point(p, q, x, e1, ell)),
    ]:
        out = torch.empty(ref.size, dtype=torch.float64, device="cuda:0")
        G.factor(kind, p, q, a1, a2, ell, out)
        got = host(out).reshape(ref.shape)
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-11 * scale, (kind, np.abs(got - ref).max() / scale)


# ---------------------------------------------------------------------------
# dense Gram and matvec
# ---------------------------------------------------------------------------
SMALL = {
    "heat1d_c1": lambda: W.heat1d_c1(),
    "advdiff_6x7": lambda: W.advdiff_c2(nt=6, nx=7, n_ic=10),
    "heat2d_3x4x3": lambda: W.heat2d_c3(nt=3, nx=4, ny=3, n_ic=4, n_bt=3, n_bs=2),
    "wave_3x4x5": lambda: W.wave2d_c4(nt=3, nx=4, ny=5, n_ic=4, n_bt=3, n_bs=2),
}

RAGGED = {
    "advdiff_37x45": lambda: W.advdiff_c2(nt=37, nx=45, n_ic=50),
    "heat2d_9x33x20": lambda: W.heat2d_c3(nt=9, nx=33, ny=20, n_ic=12, n_bt=5, n_bs=7),
    "wave_5x40x33": lambda: W.wave2d_c4(nt=5, nx=40, ny=33, n_ic=10, n_bt=4, n_bs=6),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_dense_gram_block_matches_oracle(G, name):
    p = SMALL[name]()
    ref = O.Oracle(p).gram()
    h = G.assemble(p, max_iter=8)
    try:
        n = ref.shape[0]
        out = torch.empty(n * n, dtype=torch.float64, device="cuda:0")
        G.gram_block(h, 0, n, 0, n, out)
        got = host(out).reshape(n, n)
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
        # an off-origin rectangular block
        out2 = torch.empty(7 * 5, dtype=torch.float64, device="cuda:0")
        G.gram_block(h, n - 7, 7, 3, 5, out2)
        assert np.abs(host(out2).reshape(7, 5) - ref[n - 7:, 3:8]).max() <= 1e-11 * np.abs(ref).max()
    finally:
        G.destroy(h)


@pytest.mark.parametrize("name", list(SMALL) + list(RAGGED))
@pytest.mark.parametrize("nrhs", [1, 3])
def test_fp64_matvec_matches_dense_oracle(G, name, nrhs):
    p = {**SMALL, **RAGGED}[name]()
    Gd = O.Oracle(p).gram()
    n = Gd.shape[0]
    rng = np.random.default_rng(11)
    X = rng.standard_normal((nrhs, n))
    h = G.assemble(p, max_iter=8)
    try:
        y = torch.empty(nrhs * n, dtype=torch.float64, device="cuda:0")
        G.matvec(h, dev(X.ravel()), y, nrhs=nrhs)
        Y = host(y).reshape(nrhs, n)
        for r in range(nrhs):
            ref = Gd @ X[r]
            assert relerr(Y[r], ref) <= 1e-11, (r, relerr(Y[r], ref))
    finally:
        G.destroy(h)


# ---------------------------------------------------------------------------
# solve + posterior
# ---------------------------------------------------------------------------
def _gpu_posterior(G, p, iters, tol, prec=0, grid=None, passes=2):
    h = G.assemble(p, max_iter=max(iters, 1))
    try:
        info = G.solve(h, prec=prec, tol=tol, max_iter=iters, check_every=4, reorth_passes=passes)
        axes = grid if grid is not None else p.grid
        M = int(np.prod([len(a) for a in axes]))
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, axes, mean, var)
        return host(mean), host(var), info
    finally:
        G.destroy(h)


def test_c1_mean_matches_cholesky_oracle(G):
    p = W.heat1d_c1()
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    m_ref, v_ref, _ = O.dense_posterior(o, X)
    m, v, info = _gpu_posterior(G, p, 256, 1e-10)
    assert info["rel_res"] <= 1e-8, info
    assert_close(m, m_ref, 1e-6, converged=True)
    assert np.all(v >= v_ref - 1e-9)            # combined >= mathematical variance


@pytest.mark.parametrize("k", [1, 7, 40])
@pytest.mark.parametrize("passes", [1, 2])
def test_itergp_fixed_iterations_match_oracle(G, k, passes):
    """Same IterGP recurrences for k iterations: mean and combined variance."""
    p = W.heat1d_c1()
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    S = SchurSystem(o)
    vp, D, eta, _ = O.itergp(S, k, passes=passes)
    m_ref, v_ref = two_stage_posterior(S, vp, X, D, eta)
    m, v, info = _gpu_posterior(G, p, k, 0.0, passes=passes)
    assert info["iters"] == k
    assert_close(m, m_ref, 1e-6)
    assert_close(v, v_ref, 1e-6)


def test_advdiff_small_matches_cholesky(G):
    p = W.advdiff_c2(nt=24, nx=20, n_ic=40)
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    m_ref, _, _ = O.dense_posterior(o, X)
    m, v, info = _gpu_posterior(G, p, 480, 1e-9)
    assert_close(m, m_ref, 1e-6, converged=True)


def test_wave_small_itergp_matches_oracle(G):
    p = W.wave2d_c4(nt=4, nx=6, ny=5, n_ic=6, n_bt=3, n_bs=3, grid_t=3)
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    S = SchurSystem(o)
    vp, D, eta, _ = O.itergp(S, 25, passes=2)
    m_ref, v_ref = two_stage_posterior(S, vp, X, D, eta)
    m, v, info = _gpu_posterior(G, p, 25, 0.0)
    assert info["iters"] == 25
    assert_close(m, m_ref, 1e-6)
    assert_close(v, v_ref, 1e-6)


def test_mixed_matvec_error_is_float32_sized(G):
    p = RAGGED["heat2d_9x33x20"]()
    n = p.n
    rng = np.random.default_rng(3)
    x = dev(rng.standard_normal(n))
    h = G.assemble(p, max_iter=8)
    try:
        y64 = torch.empty(n, dtype=torch.float64, device="cuda:0")
        y32 = torch.empty(n, dtype=torch.float64, device="cuda:0")
        G.matvec(h, x, y64, prec=G.PREC_FP64)
        G.matvec(h, x, y32, prec=G.PREC_MIXED)
        e = relerr(host(y32), host(y64))
        assert e <= 1e-5, e
    finally:
        G.destroy(h)


@pytest.mark.parametrize("name", ["advdiff_37x45", "wave_5x40x33"])
@pytest.mark.parametrize("nrhs", [1, 2])
def test_volume_matvec_matches_oracle(G, name, nrhs):
    p = RAGGED[name]()
    o = O.Oracle(p)
    Gv = o.volume_gram()
    Gv[np.diag_indices_from(Gv)] += o.noise_pde()
    rng = np.random.default_rng(13)
    X = rng.standard_normal((nrhs, p.n_pde))
    h = G.assemble(p, max_iter=8)
    try:
        x = dev(X.ravel())
        y = torch.empty_like(x)
        for _ in range(2):          # second call reuses the plan bound to (x, y)
            G.volume_matvec(h, x, y, nrhs=nrhs)
        Y = host(y).reshape(nrhs, -1)
        for r in range(nrhs):
            assert relerr(Y[r], Gv @ X[r]) <= 1e-11
    finally:
        G.destroy(h)


# Many right-hand sides on ragged cell counts: both mode-product stages run on
# the 64x64 kernel (>= 256 tiles) with partial edge tiles and odd numbers of
# 16-deep K chunks per segment (K = 70: 5 chunks; K = 100 per term: 7).
@pytest.mark.parametrize("nt,nx,nrhs", [(100, 70, 64), (100, 70, 65), (36, 50, 96)])
def test_batched_volume_matvec_on_ragged_tiles(G, nt, nx, nrhs):
    p = W.advdiff_c2(nt=nt, nx=nx, n_ic=40)
    o = O.Oracle(p)
    s2 = o.noise_pde()
    rng = np.random.default_rng(nt + nx + nrhs)
    X = rng.standard_normal((nrhs, p.n_pde))
    h = G.assemble(p, max_iter=8)
    try:
        x = dev(X.ravel())
        y = torch.empty_like(x)
        G.volume_matvec(h, x, y, nrhs=nrhs)
        Y = host(y).reshape(nrhs, -1)
    finally:
        G.destroy(h)
    for r in range(nrhs):
        ref = o.volume_matvec(X[r]) + s2 * X[r]
        assert relerr(Y[r], ref) <= 1e-11, (r, relerr(Y[r], ref))


@pytest.mark.parametrize("name", list(RAGGED))
def test_schur_matvec_matches_oracle(G, name):
    """Volume-system operator S = G_pp + s2 I - G_pb G_bb^{-1} G_bp: one
    right-hand side (the correction through Q = L^{-1} G_bp: factored for the
    2-D case, resident for the 3-D ones) and three (Kronecker cross blocks and
    triangular solves), against the oracle's Cholesky solve."""
    p = RAGGED[name]()
    S = SchurSystem(O.Oracle(p))
    rng = np.random.default_rng(17)
    X = rng.standard_normal((3, p.n_pde))
    h = G.assemble(p, max_iter=8)
    try:
        for nrhs in (1, 3):
            y = torch.empty(nrhs * p.n_pde, dtype=torch.float64, device="cuda:0")
            G.schur_matvec(h, dev(X[:nrhs].ravel()), y, nrhs=nrhs)
            Y = host(y).reshape(nrhs, -1)
            for r in range(nrhs):
                ref = S.matvec(X[r])
                assert relerr(Y[r], ref) <= 1e-11, (nrhs, r, relerr(Y[r], ref))
    finally:
        G.destroy(h)


def test_memory_reuse_gives_identical_results_and_releases(G):
    """Handles drawing on the per-device block cache (the default) give the
    same bits as handles with their own allocations; releasing the cache
    frees its unused blocks and later handles still work."""
    p = W.advdiff_c2(nt=24, nx=20, n_ic=40)

    def run(reuse):
        h = G.assemble(p, max_iter=64, reuse_memory=reuse)
        try:
            info = G.solve(h, tol=1e-6, max_iter=64, check_every=8)
            M = int(np.prod([len(a) for a in p.grid]))
            mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
            var = torch.empty(M, dtype=torch.float64, device="cuda:0")
            G.posterior(h, p.grid, mean, var)
            return info["iters"], host(mean), host(var)
        finally:
            G.destroy(h)

    ref = run(False)
    for _ in range(2):                     # the second run takes its blocks from the cache
        it, m, v = run(True)
        assert it == ref[0] and np.array_equal(m, ref[1]) and np.array_equal(v, ref[2])
    assert G.release_cached_memory() > 0
    assert G.release_cached_memory() == 0
    it, m, v = run(True)
    assert np.array_equal(m, ref[1])


POINT_SOLVE_CASES = {
    # n_b = 512 <= the one-workgroup limit, and 8 n_b N above the resident-Q budget:
    # one right-hand side goes through the one-workgroup refined triangular solves
    "one_workgroup_solve": (lambda: W.advdiff_c2(nt=256, nx=260, n_ic=512), 1),
    # n_b = 2112 with two right-hand sides: the point-block products are GEMV-shaped
    # (few output tiles, K = n_b > 2048) and run on the split-K GEMM
    "split_k_products": (lambda: W.heat2d_c3(nt=8, nx=16, ny=16, n_ic=24, n_bt=24, n_bs=16), 2),
}


@pytest.mark.parametrize("name", list(POINT_SOLVE_CASES))
def test_point_correction_paths_match_oracle(G, name):
    """The volume-system operator on the point-solve paths that the standard
    workloads do not reach, against the oracle's Cholesky solve."""
    make, nrhs = POINT_SOLVE_CASES[name]
    p = make()
    S = SchurSystem(O.Oracle(p))
    rng = np.random.default_rng(23)
    X = rng.standard_normal((nrhs, p.n_pde))
    h = G.assemble(p, max_iter=8)
    try:
        y = torch.empty(nrhs * p.n_pde, dtype=torch.float64, device="cuda:0")
        G.schur_matvec(h, dev(X.ravel()), y, nrhs=nrhs)
        Y = host(y).reshape(nrhs, -1)
        for r in range(nrhs):
            ref = S.matvec(X[r])
            assert relerr(Y[r], ref) <= 1e-10, (r, relerr(Y[r], ref))
    finally:
        G.destroy(h)


FACTORED_CASES = {
    # initial points pinned in time and Dirichlet points pinned in space; ragged
    # 16-index work units in both orientations
    "heat1d_21x37": lambda: W.heat1d_c1(nt=21, nx=37),
    # 150 time cells: the contraction over time takes two load batches
    "heat1d_150x10": lambda: W.heat1d_c1(nt=150, nx=10, grid_n=16),
    "advdiff_40x70": lambda: W.advdiff_c2(nt=40, nx=70, n_ic=60),
}


@pytest.mark.parametrize("name", list(FACTORED_CASES))
def test_factored_point_correction_matches_oracle(G, name):
    """One right-hand side on 2-D problems whose point groups are each pinned in
    one dimension: the point-block correction Q^T Q is applied in factored form
    (per-piece contractions, P = M^T M, two extra GEMM segments), against the
    oracle's Cholesky solve of the volume system."""
    p = FACTORED_CASES[name]()
    S = SchurSystem(O.Oracle(p))
    rng = np.random.default_rng(29)
    X = rng.standard_normal(p.n_pde)
    h = G.assemble(p, max_iter=8)
    try:
        for rep in range(2):                  # the second application reuses the built pieces
            y = torch.empty(p.n_pde, dtype=torch.float64, device="cuda:0")
            G.schur_matvec(h, dev(X), y, nrhs=1)
            assert relerr(host(y), S.matvec(X)) <= 1e-11, (rep, relerr(host(y), S.matvec(X)))
    finally:
        G.destroy(h)


def test_factored_point_correction_itergp_matches_oracle(G):
    """Early-terminated IterGP (12 iterations, two-pass projection) through the
    factored correction: mean and combined variance."""
    p = W.heat1d_c1(nt=21, nx=37)
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    S = SchurSystem(o)
    vp, D, eta, _ = O.itergp(S, 12, passes=2)
    m_ref, v_ref = two_stage_posterior(S, vp, X, D, eta)
    m, v, info = _gpu_posterior(G, p, 12, 0.0, passes=2)
    assert info["iters"] == 12
    assert_close(m, m_ref, 1e-6)
    assert_close(v, v_ref, 1e-6)
