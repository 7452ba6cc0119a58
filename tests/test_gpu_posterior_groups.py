"""The point part of the posterior variance, ||L^{-1} k_b(x)||^2 (Sec. 2.1 eq.
lin-cond-cov), is computed group by group when the point groups' tensor grids
pin a dimension (one solve per free grid coordinate of each group, the vector
formed row by row) and by the chunked product L^{-1} K_b otherwise (more than
eight groups, or grouped products that would not be cheaper).  Both agree with
the oracle's two-stage IterGP posterior at a fixed iteration count, and with
each other when the same points are split into more groups (the volume system
does not depend on the order or grouping of the points)."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import gpfvm_oracle as O
from oracle.gpfvm_oracle import SchurSystem, two_stage_posterior
from parity import assert_close

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

K = 25


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_05020_amd as G
    G.lib()
    return G


def _gpu(G, p, k):
    h = G.assemble(p, max_iter=k)
    try:
        info = G.solve(h, tol=0.0, max_iter=k, check_every=4)
        assert info["iters"] == k, info
        M = int(np.prod([len(a) for a in p.grid]))
        mean = torch.empty(M, dtype=torch.float64, device="cuda:0")
        var = torch.empty(M, dtype=torch.float64, device="cuda:0")
        G.posterior(h, p.grid, mean, var)
        torch.cuda.synchronize()
        return mean.cpu().numpy(), var.cpu().numpy()
    finally:
        G.destroy(h)


def _oracle(p, k):
    o = O.Oracle(p)
    S = SchurSystem(o)
    vp, D, eta, _ = O.itergp(S, k, passes=2)
    return two_stage_posterior(S, vp, o.grid_points(p.grid), D, eta)


def _split_first(p, parts):
    """The first group (initial data on a t = 0 grid) split along its second
    dimension into `parts` groups: the same points, more groups."""
    g0 = p.groups[0]
    vals = g0.y.reshape(g0.shape)
    new = []
    for ii in np.array_split(np.arange(g0.shape[1]), parts):
        axes = [g0.axes[0], g0.axes[1][ii], g0.axes[2]]
        new.append(W.PointGroup(axes, g0.deriv, vals[:, ii, :].ravel().copy(), g0.noise_var))
    return dataclasses.replace(p, groups=new + list(p.groups[1:]))


def _wave_small():
    return W.wave2d_c4(nt=4, nx=6, ny=5, n_ic=6, n_bt=3, n_bs=3, grid_t=3)


def test_grouped_and_chunked_point_variance_match_oracle(G):
    base = _wave_small()                      # 6 groups, each pinned in one dimension: grouped form
    split = _split_first(base, 4)             # 9 groups: the chunked product
    assert len(base.groups) == 6 and len(split.groups) == 9
    res = {}
    for name, p in (("grouped", base), ("chunked", split)):
        m_ref, v_ref = _oracle(p, K)
        m, v = _gpu(G, p, K)
        assert_close(m, m_ref, 1e-6, what=f"{name} mean")
        assert_close(v, v_ref, 1e-6, what=f"{name} var")
        res[name] = (m, v)
    assert_close(res["chunked"][0], res["grouped"][0], 1e-8, what="mean, grouped vs chunked")
    assert_close(res["chunked"][1], res["grouped"][1], 1e-8, what="var, grouped vs chunked")


def test_grouped_point_variance_with_a_group_free_in_every_dimension(G):
    """A group on a 2 x 2 x 2 grid inside the domain has no pinned dimension:
    its solved columns are indexed by the whole grid (weight 1)."""
    p = _wave_small()
    inner = W.PointGroup([np.array([0.3, 0.6]), np.array([0.35, 0.7]), np.array([0.4, 0.8])], (0, 0, 0),
                         np.zeros(8), W.NOISE_EXACT)
    p = dataclasses.replace(p, groups=list(p.groups) + [inner])
    m_ref, v_ref = _oracle(p, K)
    m, v = _gpu(G, p, K)
    assert_close(m, m_ref, 1e-6, what="mean")
    assert_close(v, v_ref, 1e-6, what="var")
