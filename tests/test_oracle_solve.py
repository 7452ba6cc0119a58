"""Pins of the oracle's posterior and solvers (Sec. 2.1, Sec. 4.1, Sec. 4.2):
textbook identities (LAPACK Cholesky, block elimination, CG at convergence),
IterGP's published properties (unit-vector actions reproduce Cholesky; the
combined variance bounds the exact one and shrinks monotonically), interpolation
in the noise-free limit, and convergence to analytic PDE solutions."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import gpfvm_oracle as O
from oracle.gpfvm_oracle import SchurSystem, two_stage_posterior


def test_dense_posterior_is_the_gaussian_conditional():
    """Compare against the joint-Gaussian conditional formed by hand from the
    joint covariance [[G, Lk],[Lk^T, k(X,X)]] with numpy's generic solve."""
    p = W.heat1d_c1(nt=4, nx=4, n_ic=6, grid_n=4)
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    m, v, _ = O.dense_posterior(o, X)
    G = o.gram()
    kb, kp = o.Lk_points(X)
    Lk = np.vstack([kb, kp])
    kxx = np.exp(-0.5 * (((X[:, None, :] - X[None, :, :]) / np.array(p.lengthscale)) ** 2).sum(-1))
    m_ref = Lk.T @ np.linalg.solve(G, p.y_obs())
    C_ref = kxx - Lk.T @ np.linalg.solve(G, Lk)
    assert np.allclose(m, m_ref, rtol=1e-9, atol=1e-10)
    assert np.allclose(v, np.diag(C_ref), rtol=1e-7, atol=1e-10)


def test_point_observations_are_interpolated():
    p = W.heat1d_c1(nt=4, nx=4, n_ic=6)
    o = O.Oracle(p)
    g = p.groups[1]                     # Dirichlet points at x = 0, noise 1e-8
    X = np.stack([m.ravel() for m in np.meshgrid(*g.axes, indexing="ij")], 1)
    m, v, _ = O.dense_posterior(o, X)
    assert np.abs(m - g.y).max() < 1e-4
    assert v.max() < 1e-7 and v.min() >= 0.0


def test_two_stage_equals_one_stage_and_unit_actions_reproduce_cholesky():
    """Sec. 4.2: conditioning on IC/BC by Cholesky first, then on the volumes,
    gives the one-stage posterior; IterGP with unit-vector actions run for
    all N iterations is a Cholesky factorisation (Wenger et al. 2022)."""
    p = W.advdiff_c2(nt=6, nx=6, n_ic=10)
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    m, v, alpha = O.dense_posterior(o, X)
    S = SchurSystem(o)
    Sd = np.stack([S.matvec(e) for e in np.eye(p.n_pde)], 1)
    vp = np.linalg.solve(Sd, S.b)
    assert np.allclose(S.full_weights(vp), alpha, rtol=1e-7, atol=1e-9 * np.abs(alpha).max())
    vu, D, eta, _ = O.itergp(S, p.n_pde, actions="unit")
    assert D.shape[1] == p.n_pde
    m2, v2 = two_stage_posterior(S, vu, X, D, eta)
    assert np.linalg.norm(m2 - m) <= 1e-8 * np.linalg.norm(m)
    assert np.linalg.norm(v2 - v) <= 1e-6 * np.linalg.norm(v)
    # and C_N is the inverse of S
    C = D @ np.diag(1 / eta) @ D.T
    assert np.allclose(C @ Sd, np.eye(p.n_pde), atol=1e-6)


def test_itergp_cg_properties():
    p = W.heat1d_c1(nt=8, nx=8, n_ic=16, grid_n=9)
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    m_ex, v_ex, _ = O.dense_posterior(o, X)
    S = SchurSystem(o)
    prev = None
    for k in (2, 5, 10, 20):
        vp, D, eta, res = O.itergp(S, k)
        m, var = two_stage_posterior(S, vp, X, D, eta)
        # combined variance >= mathematical variance (computational uncertainty >= 0)
        assert np.all(var >= v_ex - 1e-9)
        if prev is not None:
            assert np.all(var <= prev + 1e-9)       # non-increasing in the iteration count
        prev = var
    # IterGP with CG actions reproduces plain CG's iterate (same Krylov space)
    for k in (3, 7):
        vp, D, eta, _ = O.itergp(S, k)
        x_cg, _ = _cg_fixed(S, k)
        assert np.linalg.norm(vp - x_cg) <= 1e-6 * np.linalg.norm(x_cg)
    # with a tolerance, the mean converges to the Cholesky mean
    vp, D, eta, res = O.itergp(S, p.n_pde, tol=1e-10)
    m, _ = two_stage_posterior(S, vp, X)
    assert np.linalg.norm(m - m_ex) <= 1e-7 * np.linalg.norm(m_ex)


def _cg_fixed(S, k):
    b = S.b
    x = np.zeros_like(b); r = b.copy(); pp = r.copy(); rr = r @ r
    for _ in range(k):
        Ap = S.matvec(pp); a = rr / (pp @ Ap)
        x += a * pp; r -= a * Ap; rr2 = r @ r
        pp = r + rr2 / rr * pp; rr = rr2
    return x, k


def test_cg_solve_matches_cholesky():
    p = W.advdiff_c2(nt=8, nx=8, n_ic=12)
    o = O.Oracle(p)
    _, _, alpha = O.dense_posterior(o, o.grid_points(p.grid))
    S = SchurSystem(o)
    x, it = O.cg_solve(S, 1e-11, 2000)
    a2 = S.full_weights(x)
    assert np.linalg.norm(a2 - alpha) <= 1e-6 * np.linalg.norm(alpha)


def test_heat_posterior_converges_to_analytic_solution():
    """u_t = 0.1 u_xx, u(0,x) = sin(pi x), u(t,0)=u(t,1)=0 has the solution
    exp(-0.1 pi^2 t) sin(pi x).  With noise-free IC data the posterior mean's
    error must fall as the volumes are refined."""
    errs = []
    for n in (4, 8, 16):
        p = W.heat1d_c1(nt=n, nx=n, n_ic=32, grid_n=21)
        p.groups[0].y = np.sin(np.pi * p.groups[0].axes[1])
        p.groups[0].noise_var = 1e-8
        o = O.Oracle(p)
        X = o.grid_points(p.grid)
        m, _, _ = O.dense_posterior(o, X)
        u = np.exp(-0.1 * np.pi ** 2 * X[:, 0]) * np.sin(np.pi * X[:, 1])
        errs.append(np.sqrt(np.mean((m - u) ** 2)))
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1], errs
    assert errs[2] < 1e-3, errs


def test_ode_toy_fvm_converges_to_sine():
    """Fig. 'collocation vs FVM' problem: du/dx = cos x on [0, 2 pi] with
    u(0) = u(2 pi) = 0; volume data int_I cos = sin b - sin a.  Posterior mean
    -> sin x."""
    errs = []
    for n in (4, 8, 16):
        e = np.linspace(0, 2 * np.pi, n + 1)
        p = W.IBVP(name="toy", d=1, edges=[e], lengthscale=(1.0,), outputscale=1.0,
                   terms=[W.PDETerm((1,), 1.0)],
                   groups=[W.PointGroup([np.array([0.0, 2 * np.pi])], (0,), np.zeros(2), 1e-10)],
                   f_int=np.sin(e[1:]) - np.sin(e[:-1]), noise_pde=1e-10, noise_pde_relative=False,
                   grid=[np.linspace(0, 2 * np.pi, 50)])
        o = O.Oracle(p)
        X = o.grid_points(p.grid)
        m, v, _ = O.dense_posterior(o, X)
        errs.append(np.abs(m - np.sin(X[:, 0])).max())
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-3, errs


# ---------------------------------------------------------------------------
# IterGP at a fixed iteration count k << N (Sec. 4.1).  With CG actions the
# first k directions span the Krylov space K_k(S, b), and IterGP's inverse
# approximation C_k = D diag(1/eta) D^T is the S-Galerkin projector onto it:
# C_k = V (V^T S V)^{-1} V^T for any basis V, and v_k = C_k b.  The pin builds
# V by Arnoldi (twice-orthogonalised) on the dense S formed from the dense
# Gram blocks, independent of the matrix-free operator and of the recurrence.
# ---------------------------------------------------------------------------
def _dense_schur(o, p):
    G = o.gram()
    nb = p.n_b
    Gbb, Gbp, Gpp = G[:nb, :nb], G[:nb, nb:], G[nb:, nb:]
    return Gpp - Gbp.T @ np.linalg.solve(Gbb, Gbp)


def _krylov_basis(A, b, k):
    V = np.zeros((len(b), k))
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(1, k):
        w = A @ V[:, j - 1]
        for _ in range(2):
            w -= V[:, :j] @ (V[:, :j].T @ w)
        V[:, j] = w / np.linalg.norm(w)
    return V


def _galerkin_gap(itergp_fn, S, Sd, k):
    """Relative distance of (v_k, C_k) from the Krylov-Galerkin solution."""
    V = _krylov_basis(Sd, S.b, k)
    H = V.T @ Sd @ V
    Cg = V @ np.linalg.solve(H, V.T)
    xg = Cg @ S.b
    vp, D, eta = itergp_fn(S, k)[:3]
    C = D @ np.diag(1.0 / eta) @ D.T
    return (np.linalg.norm(vp - xg) / np.linalg.norm(xg), np.abs(C - Cg).max() / np.abs(Cg).max())


@pytest.mark.parametrize("passes", [1, 2])
def test_itergp_fixed_k_is_the_krylov_galerkin_projection(passes):
    p = W.heat1d_c1(nt=8, nx=8, n_ic=16, grid_n=9)
    o = O.Oracle(p)
    S = SchurSystem(o)
    Sd = _dense_schur(o, p)
    # the projected matrix V^T S V reaches cond 7e4 at k = 40: bound 1e-9 there
    for k, tol in ((1, 1e-13), (7, 1e-12), (20, 1e-11), (40, 1e-9)):
        gv, gc = _galerkin_gap(lambda S_, k_: O.itergp(S_, k_, passes=passes), S, Sd, k)
        assert gv <= tol and gc <= tol, (k, gv, gc)


def test_itergp_two_pass_variance_bounds_and_cg_iterate():
    """Two-pass IterGP at fixed k: combined variance >= the exact one and
    non-increasing in k; for small k (before plain CG loses orthogonality) the
    iterate is textbook CG's."""
    p = W.heat1d_c1(nt=8, nx=8, n_ic=16, grid_n=9)
    o = O.Oracle(p)
    X = o.grid_points(p.grid)
    _, v_ex, _ = O.dense_posterior(o, X)
    S = SchurSystem(o)
    prev = None
    for k in (2, 5, 10, 20, 40):
        vp, D, eta, _ = O.itergp(S, k, passes=2)
        _, var = two_stage_posterior(S, vp, X, D, eta)
        assert np.all(var >= v_ex - 1e-9)
        if prev is not None:
            assert np.all(var <= prev + 1e-9)
        prev = var
    for k in (1, 3, 7):
        vp, _, _, _ = O.itergp(S, k, passes=2)
        x_cg, _ = _cg_fixed(S, k)
        assert np.linalg.norm(vp - x_cg) <= 1e-12 * np.linalg.norm(x_cg)


def _itergp_second_pass_with_z(S, k):
    """A plausible slip planted in a copy of the two-pass recurrence: the
    second projection reuses z = S s instead of S d."""
    b = S.b
    n = len(b)
    v = np.zeros(n); D = np.zeros((n, k)); eta = np.zeros(k)
    for i in range(k):
        r = b - S.matvec(v) if i > 0 else b.copy()
        z = S.matvec(r)
        d = r - D[:, :i] @ ((D[:, :i].T @ z) / eta[:i]) if i > 0 else r.copy()
        if i > 0:
            d = d - D[:, :i] @ ((D[:, :i].T @ z) / eta[:i])
        eta[i] = d @ S.matvec(d)
        D[:, i] = d
        v = v + (r @ r) / eta[i] * d
    return v, D, eta


def test_galerkin_pin_detects_a_planted_projection_slip():
    p = W.heat1d_c1(nt=8, nx=8, n_ic=16, grid_n=9)
    o = O.Oracle(p)
    S = SchurSystem(o)
    Sd = _dense_schur(o, p)
    gv, gc = _galerkin_gap(_itergp_second_pass_with_z, S, Sd, 7)
    assert gv > 1e-2 and gc > 1e-2, (gv, gc)
