"""Degenerate inputs of the oracle: no IC/BC observations (an empty point
block, Sec. 2.2 stacking with an empty IC/BC set), all-zero data, a single
time cell, a single evaluation point."""
import numpy as np

import workloads as W
from oracle import gpfvm_oracle as O
from oracle.gpfvm_oracle import SchurSystem, two_stage_posterior


def no_points_with_source():
    """heat 1-D with only volume observations and a seeded source term."""
    p = W.heat1d_c1()
    p.groups = []
    vol = np.outer(np.diff(p.edges[0]), np.diff(p.edges[1])).ravel()
    p.f_int = np.random.default_rng(17).standard_normal(p.n_pde) * vol
    return p


def test_empty_point_block_two_stage_equals_dense():
    p = no_points_with_source()
    o = O.Oracle(p)
    S = SchurSystem(o)
    assert o.point_gram().shape == (0, 0) and o.cross_gram().shape == (0, p.n_pde)
    Gv = o.volume_gram() + o.noise_pde() * np.eye(p.n_pde)
    assert np.allclose(S.matvec(np.ones(p.n_pde)), Gv @ np.ones(p.n_pde), rtol=1e-12, atol=0)
    X = o.grid_points(p.grid)
    m_ref, v_ref, _ = O.dense_posterior(o, X)
    # without IC/BC data the volume system is nearly singular (the PDE alone leaves the
    # solution almost free): converge to 1e-8, the mean then matches and the combined
    # variance stays above the exact one
    vp, D, eta, _ = O.itergp(S, p.n_pde, tol=1e-8, passes=2)
    m, v = two_stage_posterior(S, vp, X, D, eta)
    assert np.linalg.norm(m - m_ref) <= 1e-6 * np.linalg.norm(m_ref)
    assert np.all(v >= v_ref - 1e-9)


def test_zero_data_gives_zero_mean_and_no_directions():
    p = W.heat1d_c1()
    for g in p.groups:
        g.y = np.zeros_like(g.y)
    o = O.Oracle(p)
    S = SchurSystem(o)
    vp, D, eta, res = O.itergp(S, 10, tol=1e-8, passes=2)
    assert D.shape[1] == 0 and res[0] == 0.0
    X = o.grid_points([np.array([0.5]), np.array([0.25, 0.75])])
    m, v = two_stage_posterior(S, vp, X, D, eta)
    assert np.all(m == 0.0)
    # no volume directions: only the point block reduces the prior
    kb, _ = o.Lk_points(X)
    Wb = np.linalg.solve(np.linalg.cholesky(o.point_gram()), kb)
    assert np.allclose(v, o.sf2 - (Wb * Wb).sum(0), rtol=0, atol=1e-12)
