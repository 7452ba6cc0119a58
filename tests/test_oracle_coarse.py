"""Pins of the oracle's coarse-scheme warm start (appendix "Multigrid
preconditioners"): conditioning exactly on nested coarse volumes, then IterGP
with CG actions on the fine volumes."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import gpfvm_oracle as O
from oracle.gpfvm_oracle import SchurSystem, two_stage_posterior


def _coarse_ibvp(p, f, noise_abs):
    """The same IBVP observed on the coarse scheme only: every f-th cell edge
    (nested refinement), volume data summed, a given absolute noise."""
    q = copy.deepcopy(p)
    q.edges = [np.asarray(e)[::k].copy() for e, k in zip(p.edges, f)]
    if p.f_int is not None:
        q.f_int = O.coarse_aggregation(p, f) @ np.asarray(p.f_int, float)
    q.noise_pde = noise_abs
    q.noise_pde_relative = False
    return q


@pytest.mark.parametrize("name,f", [("heat1d", (4, 2)), ("advdiff", (3, 5))])
def test_aggregated_fine_gram_is_the_coarse_gram(name, f):
    """eq. subdomain-partition: a coarse cell's functional is the sum of its
    fine cells', so C G_VV C^T equals the Gram the coarse scheme assembles
    from its own (coarse-edge) closed-form factors, and C L_V k(x) equals its
    cross-covariance with points."""
    p = W.heat1d_c1() if name == "heat1d" else W.advdiff_c2(nt=12, nx=10, n_ic=20)
    o = O.Oracle(p)
    C = O.coarse_aggregation(p, f)
    oc = O.Oracle(_coarse_ibvp(p, f, 0.0))
    Gf, Gc = o.volume_gram(), oc.volume_gram()
    assert np.abs(C @ Gf @ C.T - Gc).max() <= 1e-11 * np.abs(Gc).max()
    X = np.random.default_rng(0).uniform(0, 1, (7, 2))
    assert np.abs(C @ o.Lk_points(X)[1] - oc.Lk_points(X)[1]).max() <= 1e-11 * np.abs(oc.Lk_points(X)[1]).max()


def test_aggregation_matrix_structure():
    p = W.wave2d_c4(nt=4, nx=6, ny=5, n_ic=6, n_bt=3, n_bs=3, grid_t=3)
    C = O.coarse_aggregation(p, (2, 3, 5))
    assert C.shape == (2 * 2 * 1, 120)
    assert np.all(C.sum(axis=0) == 1) and np.all(C.sum(axis=1) == 2 * 3 * 5)
    # fine cell (t, x, y) = (3, 4, 2) lies in coarse cell (1, 1, 0)
    assert C[np.ravel_multi_index((1, 1, 0), (2, 2, 1)), np.ravel_multi_index((3, 4, 2), (4, 6, 5))] == 1
    with pytest.raises(ValueError):
        O.coarse_aggregation(p, (3, 3, 5))


@pytest.mark.parametrize("name,f", [("heat1d", (4, 4)), ("advdiff", (3, 5))])
def test_coarse_block_is_exact_conditioning_on_the_coarse_scheme(name, f):
    """After the coarse block alone, the two-stage posterior equals the dense
    posterior of points + coarse volumes (the coarse scheme assembled on its
    own, with the aggregated fine noise)."""
    p = W.heat1d_c1() if name == "heat1d" else W.advdiff_c2(nt=12, nx=10, n_ic=20)
    o = O.Oracle(p)
    S = SchurSystem(o)
    C = O.coarse_aggregation(p, f)
    v, D, eta, _ = O.itergp_coarse(S, C, 0)
    assert D.shape[1] == C.shape[0] and np.allclose(eta, 1.0)
    X = o.grid_points(p.grid)
    m, var = two_stage_posterior(S, v, X, D, eta)
    oc = O.Oracle(_coarse_ibvp(p, f, o.noise_pde() * int(np.prod(f))))
    m_ref, v_ref, _ = O.dense_posterior(oc, X)
    assert np.linalg.norm(m - m_ref) <= 1e-8 * np.linalg.norm(m_ref)
    assert np.abs(var - v_ref).max() <= 1e-8


def test_coarse_then_cg_reaches_the_exact_posterior_and_saves_iterations():
    p = W.advdiff_c2(nt=12, nx=10, n_ic=20)
    o = O.Oracle(p)
    S = SchurSystem(o)
    C = O.coarse_aggregation(p, (3, 5))
    X = o.grid_points(p.grid)
    m_ref, v_ref, _ = O.dense_posterior(o, X)
    v, D, eta, _ = O.itergp_coarse(S, C, p.n_pde - C.shape[0], passes=2)
    assert D.shape[1] == p.n_pde
    m, var = two_stage_posterior(S, v, X, D, eta)
    assert np.linalg.norm(m - m_ref) <= 1e-6 * np.linalg.norm(m_ref)
    assert np.abs(var - v_ref).max() <= 1e-6
    # to 1e-6 on the fine system: fewer CG iterations after the coarse block
    _, _, _, r_plain = O.itergp(S, p.n_pde, tol=1e-6, passes=2)
    _, _, _, r_coarse = O.itergp_coarse(S, C, p.n_pde, tol=1e-6, passes=2)
    assert len(r_coarse) < len(r_plain), (len(r_coarse), len(r_plain))
