"""Mixed-precision path and the plain CG method, through the C-ABI.

Mixed path (GPFVM_PREC_MIXED): the volume Gram (Sec. 4.1 eq.
kronecker-structure) runs in low precision -- float32 on the float32 matrix
cores, or float32 tensors split into three bfloat16 slices on the bfloat16
matrix cores (float32 accuracy) -- inside float64 iterative refinement:
blocks of low-precision IterGP iterations (Sec. 4.1), each started from the
float64 residual b - S v and re-stabilised in float64 (float64 S D,
S-conjugation against the stored directions, the small projected Cholesky).
Tolerance 1e-4 against the float64 oracle for mean and combined variance:
the low-precision operator changes which Krylov space the blocks explore by
about its rounding (1e-7 relative), which a CPU emulation of the scheme with
the same slice arithmetic puts at 1e-6 (40 iterations) and 3e-5 (120
iterations) on advection-diffusion 128 x 128.

CG (GPFVM_METHOD_CG): O(N) state, no stored directions (Sec. 4.1, iterative
techniques); compared with the oracle's textbook CG and with Cholesky."""
import numpy as np
import pytest

import workloads as W
from parity import assert_close, relerr
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


RAGGED = {
    "advdiff_37x45": lambda: W.advdiff_c2(nt=37, nx=45, n_ic=50),
    "wave_5x40x33": lambda: W.wave2d_c4(nt=5, nx=40, ny=33, n_ic=10, n_bt=4, n_bs=6),
}


@pytest.mark.parametrize("tile", [0, 1])
@pytest.mark.parametrize("name", list(RAGGED))
@pytest.mark.parametrize("nrhs", [1, 64])
def test_low_precision_volume_matvec_is_float32_accurate(G, tile, name, nrhs):
    """Both tile formats against the oracle's float64 Kronecker matvec over the
    quadrature factors: float32-sized error (ragged 32x32 tiles with one rhs,
    64x64 tiles with 64)."""
    p = RAGGED[name]()
    o = O.Oracle(p)
    s2 = o.noise_pde()
    rng = np.random.default_rng(41 + nrhs)
    X = rng.standard_normal((nrhs, p.n_pde))
    h = G.assemble(p, max_iter=8, tile=tile)
    try:
        x = torch.as_tensor(X.ravel(), device="cuda:0")
        y = torch.empty_like(x)
        G.volume_matvec(h, x, y, nrhs=nrhs, prec=G.PREC_MIXED)
        Y = host(y).reshape(nrhs, -1)
    finally:
        G.destroy(h)
    for r in (0, nrhs - 1):
        ref = o.volume_matvec(X[r]) + s2 * X[r]
        e = relerr(Y[r], ref)
        assert 1e-12 < e <= 2e-6, (r, e)          # float32 accuracy, and not the float64 plan


@pytest.fixture(scope="module")
def c2():
    p = W.advdiff_c2()
    o = O.Oracle(p)
    S = SchurSystem(o)
    X = o.grid_points(p.grid)
    idx = np.sort(np.random.default_rng(2).choice(len(X), size=384, replace=False))
    return p, o, S, X, idx


def _mixed(G, p, k, tol, tile, block=32, grid_var=True):
    h = G.assemble(p, max_iter=k, tile=tile)
    try:
        info = G.solve(h, prec=G.PREC_MIXED, tile=tile, tol=tol, max_iter=k, block=block, check_every=8)
        M = int(np.prod([len(a) for a in p.grid]))
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean, var)
        return info, host(mean), host(var)
    finally:
        G.destroy(h)


@pytest.mark.parametrize("tile,k", [(1, 40), (1, 120), (0, 40)])
def test_mixed_fixed_iterations_match_oracle(G, c2, tile, k):
    """Advection-diffusion 128 x 128 (the benchmark's small configuration):
    k mixed iterations in blocks of 32 against k float64 IterGP iterations of
    the oracle, mean and combined variance within 1e-4.  (The float32-MFMA
    tiles accumulate in a different order than the split-bfloat16 ones; at
    120 iterations their mean lands at 9e-5 L2 / 1.3e-4 pointwise, so that
    case is left to the split tiles.)"""
    p, o, S, X, idx = c2
    vp, D, eta, _ = O.itergp(S, k, passes=2)
    m_ref, v_ref = two_stage_posterior(S, vp, X[idx], D, eta)
    info, m, v = _mixed(G, p, k, 0.0, tile)
    print(f"tile {tile}, k {k}: {info}", flush=True)
    assert info["iters"] == k and info["outer"] == (k + 31) // 32, info
    assert_close(m[idx], m_ref, 1e-4, what="mean")
    assert_close(v[idx], v_ref, 1e-4, what="var")


def test_mixed_converges_to_the_oracle_mean(G, c2):
    """To 1e-8 with split-bfloat16 tiles: the float64 residual meets the
    tolerance, the mean equals the oracle's converged mean (two solves stopped
    at a residual tolerance), and the combined variance bounds the exact
    (Cholesky) posterior variance from above."""
    p, o, S, X, idx = c2
    vp, D, eta, _ = O.itergp(S, 2000, tol=1e-8, passes=2)
    m_ref, _ = two_stage_posterior(S, vp, X[idx])
    _, v_exact, _ = O.dense_posterior(o, X[idx])
    info, m, v = _mixed(G, p, 2048, 1e-8, 1)
    print(f"mixed to 1e-8: {info}; float64 oracle IterGP: {D.shape[1]} iterations", flush=True)
    assert info["rc"] == G.OK and info["rel_res"] <= 1e-8, info
    assert info["iters"] <= 1.25 * D.shape[1], (info["iters"], D.shape[1])
    assert_close(m[idx], m_ref, 1e-6, what="mean", converged=True)
    assert np.all(v[idx] >= v_exact - 1e-9), float(np.min(v[idx] - v_exact))


def _cg_gpu(G, p, tol, iters):
    h = G.assemble(p, max_iter=1)
    try:
        info = G.solve(h, tol=tol, max_iter=iters, method=G.METHOD_CG, check_every=16)
        alpha = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
        G.weights(h, alpha)
        M = int(np.prod([len(a) for a in p.grid]))
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean)
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        with pytest.raises(G.GpfvmError) as e:                      # the variance needs the directions
            G.posterior(h, p.grid, mean, var)
        assert e.value.code == G.E_STATE
        with pytest.raises(G.GpfvmError):                           # CG does not resume
            G.solve(h, tol=tol, max_iter=10, method=G.METHOD_CG, resume=True, raise_on_noconv=True)
        return info, host(alpha)[p.n_b:], host(mean)
    finally:
        G.destroy(h)


CG_CASES = {
    # factored point correction (2-D, one initial group)
    "advdiff_24x20": lambda: W.advdiff_c2(nt=24, nx=20, n_ic=40),
    # row-streaming triangular point solves (3-D, n_b = 768 > 512)
    "heat2d_request_16x16x16": lambda: W.heat2d_request(16, 16, seed=4244),
}


@pytest.mark.parametrize("name", list(CG_CASES))
def test_cg_method_converges_like_textbook_cg(G, name):
    """Plain CG keeps no directions and so no reorthogonalisation: its
    iterates are chaotic in rounding on these systems (on the CPU, a 1e-15
    relative perturbation of the operator moves the 30-iteration posterior
    mean by 0.1-0.8%), so it is compared where that does not matter: with PDE
    noise at 1e-2 of the mean diagonal (better conditioned than the
    benchmark's 1e-6, where plain CG stalls in float64 on both sides), the
    iteration count of textbook CG to 1e-10 and the posterior mean of the
    Cholesky solve."""
    p = CG_CASES[name]()
    p.noise_pde = 1e-2
    o = O.Oracle(p)
    S = SchurSystem(o)
    _, it_ref = O.cg_solve(S, 1e-10, 5000)
    m_chol, _, _ = O.dense_posterior(o, o.grid_points(p.grid))
    info, _, m = _cg_gpu(G, p, 1e-10, 5000)
    assert it_ref < 5000 and info["rc"] == G.OK and info["rel_res"] <= 1e-9, (info, it_ref)
    assert abs(info["iters"] - it_ref) <= 3 + 0.03 * it_ref, (info, it_ref)
    assert_close(m, m_chol, 1e-6, what="mean", converged=True)


def test_matvec_float32_io(G):
    """gpfvm_matvec with float32 input and output: the float64 product of the
    widened input, rounded to float32."""
    p = W.heat2d_c3(nt=9, nx=33, ny=20, n_ic=12, n_bt=5, n_bs=7)
    rng = np.random.default_rng(43)
    x = rng.standard_normal(p.n).astype(np.float32)
    h = G.assemble(p, max_iter=8)
    try:
        y32 = torch.empty(p.n, dtype=torch.float32, device="cuda:0")
        G.matvec(h, torch.as_tensor(x, device="cuda:0"), y32)
        y64 = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
        G.matvec(h, torch.as_tensor(x.astype(np.float64), device="cuda:0"), y64)
        ref = host(y64)
        assert np.array_equal(host(y32), ref.astype(np.float32))
    finally:
        G.destroy(h)
