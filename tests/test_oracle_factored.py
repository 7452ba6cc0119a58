"""The factored point correction of a one-rhs volume operator, checked on the
CPU against the plain Cholesky form.

For a 2-D problem whose point groups are each pinned in one dimension (initial
data at t = 0, Dirichlet edges at x = 0 and 1), the cross block of each group
and PDE term is the outer product of its point-cell factors over the two
dimensions (Sec. 3.2, the operator distributes over the 1-D factors).  Then

    G_pb G_bb^{-1} G_bp x = sum_r q_r (x) (P w)_r,
    w_r = x contracted with q_r over the pinned dimension,
    P = M^T M,  M = L^{-1} [Gf_0 | Gf_1 | ...],  G_bb = L L^T,

which is the form the GPU operator applies.  The reference side uses the
oracle's dense blocks and LAPACK solves only."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import gpfvm_oracle as O


def _pieces(o, p):
    """(pinned dim, q_r, Gf_r) for every (group, PDE term)."""
    nb = sum(g.size for g in p.groups)
    out, off = [], 0
    for g in p.groups:
        pdim = 0 if len(g.axes[0]) == 1 else 1
        assert len(g.axes[pdim]) == 1, "the group must be pinned in one dimension"
        f = 1 - pdim
        for t in p.terms:
            assert not t.cellwise
            mats = o._group_cell_mats(g, g.deriv, t.alpha)   # per dim: points x cells
            q = mats[pdim][0]
            gf = np.zeros((nb, p.ncell[f]))
            gf[off:off + g.size] = o.sf2 * t.coef * mats[f]
            out.append((pdim, q, gf))
        off += g.size
    return out


@pytest.mark.parametrize("make", [lambda: W.heat1d_c1(nt=11, nx=13),
                                  lambda: W.heat1d_c1(nt=5, nx=29, n_ic=12),
                                  lambda: W.advdiff_c2(nt=9, nx=17, n_ic=20)])
def test_factored_point_correction_equals_cholesky_form(make):
    p = make()
    o = O.Oracle(p)
    n0, n1 = p.ncell
    Gbb, Gbp = o.point_gram(), o.cross_gram()
    x = np.random.default_rng(3).standard_normal(p.n_pde)
    ref = Gbp.T @ sla.cho_solve(sla.cho_factor(Gbb, lower=True), Gbp @ x)

    # the cross block is the sum of the pieces' outer products
    pcs = _pieces(o, p)
    G_sum = np.zeros_like(Gbp)
    for pdim, q, gf in pcs:
        G_sum += (np.einsum("i,bc->bic", q, gf) if pdim == 0 else np.einsum("bi,c->bic", gf, q)).reshape(Gbp.shape)
    assert np.abs(G_sum - Gbp).max() <= 1e-14 * np.abs(Gbp).max()

    L = np.linalg.cholesky(Gbb)
    M = np.hstack([sla.solve_triangular(L, gf, lower=True) for _, _, gf in pcs])
    P = M.T @ M
    X = x.reshape(n0, n1)
    w = np.concatenate([q @ X if pdim == 0 else X @ q for pdim, q, _ in pcs])
    v = P @ w
    out, a = np.zeros((n0, n1)), 0
    for pdim, q, gf in pcs:
        vr = v[a:a + gf.shape[1]]
        a += gf.shape[1]
        out += np.outer(q, vr) if pdim == 0 else np.outer(vr, q)
    assert np.linalg.norm(out.ravel() - ref) <= 1e-10 * np.linalg.norm(ref), \
        np.linalg.norm(out.ravel() - ref) / np.linalg.norm(ref)
