"""GPU parity of systems: several outputs with independent priors and several
equations per cell (Sec. 3.3 eq. multioutput-cov-def), the linearised
shallow-water equations with per-cell depth and radiation boundary rows
(appendix "Tsunami propagation", eq. sw1 to sw3), through the C-ABI against
the float64 oracle.

Tolerances as in the single-output parity tests: Gram entries and matvecs are
closed forms (1e-11 of the matrix scale, relative), posterior mean and
combined variance after the same number of IterGP iterations 1e-6 (L2 and
element-wise, each output against its own prior variance)."""
import numpy as np
import pytest

import workloads as W
from oracle import gpfvm_oracle as O
from oracle.gpfvm_oracle import SchurSystem, two_stage_posterior
from parity import assert_close
from test_oracle_multioutput import _pair_system, _rotated

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


def _sw_tiny():
    return W.shallow_water(nt=3, nx=4, ny=5, n_icx=3, n_icy=4, n_bt=2, n_bx=2, n_by=3, grid_t=2)


def _sw_se():
    return W.shallow_water(nt=2, nx=3, ny=4, n_icx=2, n_icy=3, n_bt=2, n_bx=2, n_by=2, kernel=0, grid_t=2,
                           lengthscale=(0.3, 0.2, 0.25), f_cor=0.7, drag=0.3, out_scale=(1.0, 1.7, 0.6))


def _sw1d(nt=6, nx=10):
    """1-D linearised shallow water in (t, x): h_t + H u_x = 0, u_t + g h_x + k u = 0
    with per-cell depth H (the 2-D pre-summed plan path with scaling at block
    offsets) and radiation rows h_t -/+ c h_x = 0 at x = 0 and 1 whose wave
    speed enters as a weight along t."""
    xc = W.centres(nx)
    H = 0.3 + 0.7 * np.exp(-((xc - 0.3) / 0.2) ** 2)
    cellH = np.broadcast_to(H[None, :], (nt, nx)).ravel().copy()
    xi, tb = W.centres(8), W.centres(5)
    h0 = np.exp(-0.5 * ((xi - 0.5) / 0.1) ** 2)
    groups = [W.PointGroup([np.array([0.0]), xi], (0, 0), h0, 1e-8, out=0),
              W.PointGroup([np.array([0.0]), xi.copy()], (0, 0), np.zeros(8), 1e-8, out=1)]
    for edge, sign, c in ((0.0, -1.0, np.sqrt(H[0])), (1.0, 1.0, np.sqrt(H[-1]))):
        groups.append(W.PointGroup([tb.copy(), np.array([edge])], (1, 0), np.zeros(5), 1e-8,
                                   terms=[W.PointTerm((1, 0), 1.0, 0),
                                          W.PointTerm((0, 1), sign, 0, [np.full(5, c), None])]))
    terms = [W.PDETerm((1, 0), 1.0, False, 0, 0), W.PDETerm((0, 1), 1.0, True, 1, 0),
             W.PDETerm((1, 0), 1.0, False, 1, 1), W.PDETerm((0, 1), 1.0, False, 0, 1),
             W.PDETerm((0, 0), 0.1, False, 1, 1)]
    return W.IBVP(name="sw1d", d=2, edges=[W.uniform_edges(0, 1, nt), W.uniform_edges(0, 1, nx)],
                  lengthscale=(0.3, 0.15), outputscale=1.0, terms=terms, groups=groups, cell_coef=cellH,
                  noise_pde=1e-6, grid=[W.centres(3), W.centres(12)], kernel=(3, 3), nout=2, neq=2,
                  out_scale=(1.0, 1.5))


SYSTEMS = {
    "sw1d_cellwise_2d": _sw1d,
    "sw_matern52": _sw_tiny,
    "sw_se": _sw_se,
    "decoupled_pair_2d": lambda: _pair_system()[2],
    "rotated_2d": lambda: _rotated()[2],
}


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_dense_gram_of_system_matches_oracle(G, name):
    p = SYSTEMS[name]()
    ref = O.Oracle(p).gram()
    h = G.assemble(p, max_iter=8)
    try:
        n = ref.shape[0]
        out = torch.empty(n * n, dtype=torch.float64, device="cuda:0")
        G.gram_block(h, 0, n, 0, n, out)
        got = host(out).reshape(n, n)
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
    finally:
        G.destroy(h)


@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("nrhs", [1, 3])
def test_system_matvec_matches_oracle(G, name, nrhs):
    """The whole Gram as Kronecker plans: per-equation volume blocks, cross
    blocks per (point term, PDE term) pair, the point block."""
    p = SYSTEMS[name]()
    Gd = O.Oracle(p).gram()
    n = Gd.shape[0]
    X = np.random.default_rng(21).standard_normal((nrhs, n))
    h = G.assemble(p, max_iter=8)
    try:
        y = torch.empty(nrhs * n, dtype=torch.float64, device="cuda:0")
        G.matvec(h, dev(X.ravel()), y, nrhs=nrhs)
        Y = host(y).reshape(nrhs, n)
        for r in range(nrhs):
            ref = Gd @ X[r]
            assert np.linalg.norm(Y[r] - ref) <= 1e-11 * np.linalg.norm(ref), r
    finally:
        G.destroy(h)


def _gpu_post(G, p, k, grid):
    M = int(np.prod([len(a) for a in grid]))
    h = G.assemble(p, max_iter=k)
    try:
        info = G.solve(h, tol=0.0, max_iter=k, check_every=4)
        assert info["iters"] == k, info
        mean = torch.empty(p.nout * M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(p.nout * M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, grid, mean, var)
        return host(mean).reshape(p.nout, M), host(var).reshape(p.nout, M)
    finally:
        G.destroy(h)


def _oracle_post(p, k, grid):
    o = O.Oracle(p)
    S = SchurSystem(o)
    vp, D, eta, _ = O.itergp(S, k, passes=2)
    X = o.grid_points(grid)
    out = [two_stage_posterior(S, vp, X, D, eta, out=j) for j in range(p.nout)]
    return np.stack([m for m, _ in out]), np.stack([v for _, v in out])


def _compare(G, p, k, grid=None):
    grid = p.grid if grid is None else grid
    m, v = _gpu_post(G, p, k, grid)
    mr, vr = _oracle_post(p, k, grid)
    for j, sf in enumerate(p.output_scales()):
        assert_close(m[j], mr[j], 1e-6, sf2=sf, what=f"mean of output {j}")
        assert_close(v[j], vr[j], 1e-6, sf2=sf, what=f"var of output {j}")
        assert np.all(v[j] <= sf * (1 + 1e-12)), j


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_system_posterior_after_fixed_iterations_matches_oracle(G, name):
    _compare(G, SYSTEMS[name](), 12)


def test_shallow_water_medium_posterior_matches_oracle(G):
    """12 x 16 x 20 cells (3 x 3840 volume observations), 40 iterations."""
    p = W.shallow_water(nt=12, nx=16, ny=20, n_icx=8, n_icy=10, n_bt=6, n_bx=4, n_by=5, grid_t=3)
    _compare(G, p, 40)


def test_shallow_water_row_streaming_point_block_matches_oracle(G):
    """n_b = 2340 > 512 points and 8 n_b N > 256 MiB: the point correction of every
    iteration takes the row-streaming triangular passes."""
    p = W.shallow_water(nt=10, nx=30, ny=40, n_icx=20, n_icy=25, n_bt=12, n_bx=15, n_by=20, grid_t=2)
    assert p.n_b > 512 and 8 * p.n_b * p.n_pde > 256 * 2 ** 20, (p.n_b, p.n_pde)
    grid = [W.centres(2), W.centres(9), W.centres(11)]
    _compare(G, p, 10, grid)


def test_system_is_refused_where_single_output_only(G):
    p = _sw_tiny()
    h = G.assemble(p, max_iter=8)
    try:
        with pytest.raises(G.GpfvmError) as e:
            G.solve(h, tol=1e-6, max_iter=8, prec=G.PREC_MIXED)
        assert e.value.code == G.E_INVALID
    finally:
        G.destroy(h)


def test_system_volume_matvecs_and_plain_cg(G):
    """The volume-only matvec and its allocation-free variant against the
    oracle's volume block; plain CG (mean only) against the dense posterior of
    every output, at PDE noise 1e-2 of the mean diagonal where CG converges
    without reorthogonalisation."""
    p = _sw_tiny()
    p.noise_pde = 1e-2
    o = O.Oracle(p)
    Gv = o.volume_gram() + o.noise_pde() * np.eye(p.n_pde)
    x = np.random.default_rng(5).standard_normal(p.n_pde)
    ref = Gv @ x
    h = G.assemble(p, max_iter=8)
    try:
        for fn in (G.volume_matvec, G.volume_matvec_noalloc):
            y = torch.empty(p.n_pde, dtype=torch.float64, device="cuda:0")
            fn(h, dev(x), y)
            assert np.linalg.norm(host(y) - ref) <= 1e-11 * np.linalg.norm(ref), fn.__name__
        info = G.solve(h, tol=1e-10, max_iter=2000, method=G.METHOD_CG)
        assert info["rc"] == G.OK, info
        M = int(np.prod([len(a) for a in p.grid]))
        mean = torch.empty(p.nout * M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean)
        m = host(mean).reshape(p.nout, M)
    finally:
        G.destroy(h)
    X = o.grid_points(p.grid)
    for j, sf in enumerate(p.output_scales()):
        mr, _, _ = O.dense_posterior(o, X, out=j)
        assert_close(m[j], mr, 1e-6, sf2=sf, what=f"CG mean of output {j}", converged=True)


def test_system_without_point_observations(G):
    """No initial or boundary points: the volume system is the whole Gram (with
    a seeded source term, as zero data would give no directions at all)."""
    p = _sw_tiny()
    p.groups = []
    p.f_int = np.random.default_rng(9).standard_normal(p.n_pde) * 1e-3
    _compare(G, p, 12)
