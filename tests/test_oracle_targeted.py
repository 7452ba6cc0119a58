"""Pins of the oracle's targeted uncertainty reduction (appendix "Targeted
uncertainty reduction"): IterGP whose actions are residuals of L k(X~) beta
with respect to the current inverse approximation."""
import numpy as np
import pytest

import workloads as W
from oracle import gpfvm_oracle as O
from oracle.gpfvm_oracle import SchurSystem, two_stage_posterior


def _setup():
    p = W.heat1d_c1()
    o = O.Oracle(p)
    S = SchurSystem(o)
    return p, o, S


def _textbook_cg_residuals(A, b, k):
    x = np.zeros_like(b); r = b.copy(); d = r.copy(); out = [np.linalg.norm(r)]
    for _ in range(k - 1):
        Ad = A(d)
        a = (r @ r) / (d @ Ad)
        x = x + a * d
        r_new = r - a * Ad
        d = r_new + (r_new @ r_new) / (r @ r) * d
        r = r_new
        out.append(np.linalg.norm(r))
    return np.array(out)


def test_fixed_weights_implement_cg_on_that_right_hand_side():
    """With one fixed beta the action residuals b - S C_i b are exactly the
    residuals of CG on S x = b (the appendix's statement), for both
    projection variants, started from an empty inverse approximation."""
    p, o, S = _setup()
    X = np.array([[0.7, 0.3]])
    KS = O.schur_cross(S, X)
    k = 12
    ref = _textbook_cg_residuals(S.matvec, KS[:, 0], k)
    for passes in (1, 2):
        _, _, _, res = O.itergp_targeted(S, np.zeros(p.n_pde), np.zeros((p.n_pde, 0)), np.zeros(0), KS,
                                         np.ones((k, 1)), passes=passes)
        assert np.all(np.abs(res - ref) <= 1e-8 * ref[0]), (passes, res / ref)


def test_targeted_variance_decreases_and_n_iterations_are_exact():
    p, o, S = _setup()
    grid = [np.linspace(0.6, 0.9, 3), np.linspace(0.2, 0.8, 4)]
    Xt = o.grid_points(grid)
    KS = O.schur_cross(S, Xt)
    vp, D, eta, _ = O.itergp(S, 20, passes=2)
    betas = np.random.default_rng(3).dirichlet(np.ones(len(Xt)), size=p.n_pde - 20)
    v2, D2, e2, _ = O.itergp_targeted(S, vp, D, eta, KS, betas, passes=2)
    prev = two_stage_posterior(S, vp, Xt, D, eta)[1]
    for k in (5, 20, 60):                         # combined variance non-increasing
        var = two_stage_posterior(S, vp, Xt, D2[:, :20 + k], e2[:20 + k])[1]
        assert np.all(var <= prev + 1e-12)
        prev = var
    Xg = o.grid_points(p.grid)
    m_ref, v_ref, _ = O.dense_posterior(o, Xg)
    m, v = two_stage_posterior(S, v2, Xg, D2, e2)
    assert D2.shape[1] == p.n_pde
    assert np.linalg.norm(m - m_ref) <= 1e-6 * np.linalg.norm(m_ref)
    assert np.abs(v - v_ref).max() <= 1e-6


# ---------------------------------------------------------------------------
# schur_cross: K_S(X) = Cov(L_V u, u(X) | IC/BC points).  Block elimination of
# the joint Gaussian conditional (the identity the two-stage solve of Sec. 4.2
# rests on) fixes it through the full posterior covariance and mean:
#   Cov(u(X) | all) = Cov(u(X) | points) - K_S^T S^{-1} K_S,
#   E(u(X) | all)   = E(u(X) | points)   + K_S^T S^{-1} (y_p - G_pb G_bb^{-1} y_b),
# with every other quantity formed densely from the Gram blocks and the kernel.
# The mean is linear in K_S, so it also fixes the sign.
# ---------------------------------------------------------------------------
def _block_elimination_gaps(KS_fn):
    p = W.advdiff_c2(nt=8, nx=9, n_ic=12)
    o = O.Oracle(p)
    S = SchurSystem(o)
    X = o.grid_points([np.linspace(0, 1, 5), np.linspace(0, 1, 6)])
    G = o.gram()
    nb = p.n_b
    Gbb, Gbp, Gpp = G[:nb, :nb], G[:nb, nb:], G[nb:, nb:]
    y = p.y_obs()
    kb, kp = o.Lk_points(X)
    Lk = np.vstack([kb, kp])
    ell = np.array(p.lengthscale)
    kxx = o.sf2 * np.exp(-0.5 * (((X[:, None, :] - X[None, :, :]) / ell) ** 2).sum(-1))
    cov_all = kxx - Lk.T @ np.linalg.solve(G, Lk)
    mean_all = Lk.T @ np.linalg.solve(G, y)
    cov_pts = kxx - kb.T @ np.linalg.solve(Gbb, kb)
    mean_pts = kb.T @ np.linalg.solve(Gbb, y[:nb])
    Sd = Gpp - Gbp.T @ np.linalg.solve(Gbb, Gbp)
    b = y[nb:] - Gbp.T @ np.linalg.solve(Gbb, y[:nb])
    KS = KS_fn(S, X)
    cov_gap = np.abs(cov_pts - KS.T @ np.linalg.solve(Sd, KS) - cov_all).max() / np.abs(cov_all).max()
    mean_gap = np.abs(mean_pts + KS.T @ np.linalg.solve(Sd, b) - mean_all).max() / np.abs(mean_all).max()
    return cov_gap, mean_gap


def test_schur_cross_is_the_conditioned_cross_covariance():
    cov_gap, mean_gap = _block_elimination_gaps(O.schur_cross)
    assert cov_gap <= 1e-12 and mean_gap <= 1e-12, (cov_gap, mean_gap)


def _planted(sign, solve, flip=1.0):
    """Copies of schur_cross with one plausible slip each (test of the pin)."""
    def fn(S, X):
        kb, kp = S.o.Lk_points(X)
        W_ = S.bb_solve(kb) if solve == "solve" else S.bb_lsolve(kb)
        return flip * (kp + sign * np.stack([S.o.cross_rmatvec(c) for c in W_.T], axis=1))
    return fn


@pytest.mark.parametrize("slip", ["plus", "lsolve", "negated"])
def test_schur_cross_pin_detects_planted_slips(slip):
    fn = {"plus": _planted(+1, "solve"), "lsolve": _planted(-1, "lsolve"),
          "negated": _planted(-1, "solve", flip=-1.0)}[slip]
    cov_gap, mean_gap = _block_elimination_gaps(fn)
    assert max(cov_gap, mean_gap) > 1e-2, (slip, cov_gap, mean_gap)
