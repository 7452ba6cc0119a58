"""Pins of the oracle's Gram assembly (Sec. 3.2 eq. LkL, Sec. 4.1
eq. kronecker-structure, Sec. 2.2 IBVP stacking) against brute-force
full-dimensional quadrature whose derivatives come from automatic
differentiation of the product kernel -- no 1-D factor, no Fubini, no
Kronecker product is used on the reference side."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import gpfvm_oracle as O


def _kernel(x, x2, ell):
    # x, x2: (M, d) tensors; product SE kernel
    z = ((x - x2) / torch.tensor(ell, dtype=torch.float64)) ** 2
    return torch.exp(-0.5 * z.sum(dim=1))


def _apply_op(f_of_xy, x, x2, terms1, terms2):
    """sum_{a,a'} c_a c_a' d^a_x d^{a'}_{x2} f at every row (autograd)."""
    out = torch.zeros(x.shape[0], dtype=torch.float64)
    for (a1, c1) in terms1:
        for (a2, c2) in terms2:
            xx = x.clone().requires_grad_(True)
            yy = x2.clone().requires_grad_(True)
            val = f_of_xy(xx, yy)
            for dim, order in enumerate(a1):
                for _ in range(order):
                    val = torch.autograd.grad(val.sum(), xx, create_graph=True)[0][:, dim]
            for dim, order in enumerate(a2):
                for _ in range(order):
                    val = torch.autograd.grad(val.sum(), yy, create_graph=True)[0][:, dim]
            out = out + c1 * c2 * val.detach()
    return out


def _gauss(lo, hi, n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (hi - lo) * x + 0.5 * (hi + lo), 0.5 * (hi - lo) * w


def _box_rule(box, n):
    pts, wts = zip(*[_gauss(a, b, n) for (a, b) in box])
    mesh = np.meshgrid(*pts, indexing="ij")
    wm = np.meshgrid(*wts, indexing="ij")
    X = np.stack([m.ravel() for m in mesh], 1)
    w = np.prod(np.stack([m.ravel() for m in wm], 1), axis=1)
    return X, w


def _brute_volume_pair(box1, box2, ell, terms, n=14, cc=(1.0, 1.0)):
    X1, w1 = _box_rule(box1, n)
    X2, w2 = _box_rule(box2, n)
    A = np.repeat(X1, len(X2), 0); B = np.tile(X2, (len(X1), 1))
    wt = np.repeat(w1, len(w2)) * np.tile(w2, len(w1))
    t1 = [(a, c * (cc[0] if cw else 1.0)) for (a, c, cw) in terms]
    t2 = [(a, c * (cc[1] if cw else 1.0)) for (a, c, cw) in terms]
    f = lambda x, y: _kernel(x, y, ell)
    vals = _apply_op(f, torch.from_numpy(A), torch.from_numpy(B), t1, t2).numpy()
    return float((vals * wt).sum())


def _small_heat():
    return W.heat1d_c1(nt=2, nx=3, n_ic=4, grid_n=5)


def _cells(ibvp):
    idx = np.indices(ibvp.ncell).reshape(ibvp.d, -1).T
    return [[(ibvp.edges[i][j[i]], ibvp.edges[i][j[i] + 1]) for i in range(ibvp.d)] for j in idx]


def _terms(ibvp):
    return [(t.alpha, t.coef, t.cellwise) for t in ibvp.terms]


def test_volume_gram_matches_bruteforce_heat():
    p = _small_heat()
    o = O.Oracle(p)
    G = o.volume_gram()
    cells = _cells(p)
    for (i, j) in [(0, 0), (0, 1), (1, 4), (5, 2)]:
        ref = _brute_volume_pair(cells[i], cells[j], p.lengthscale, _terms(p))
        assert abs(G[i, j] - ref) <= 1e-10 * max(1.0, abs(ref)), (i, j, G[i, j], ref)


def test_volume_gram_matches_bruteforce_advection():
    p = W.advdiff_c2(nt=2, nx=3, n_ic=4)
    o = O.Oracle(p)
    G = o.volume_gram()
    cells = _cells(p)
    for (i, j) in [(0, 0), (0, 1), (2, 3), (4, 1)]:
        ref = _brute_volume_pair(cells[i], cells[j], p.lengthscale, _terms(p))
        assert abs(G[i, j] - ref) <= 1e-9 * max(1.0, abs(ref)), (i, j, G[i, j], ref)


def test_volume_gram_cellwise_coefficient_3d():
    """Wave operator with per-cell c^2 (appendix, variable bathymetry)."""
    p = W.wave2d_c4(nt=2, nx=2, ny=2, n_ic=2, n_bt=2, n_bs=1, grid_t=2)
    # narrow cells relative to the lengthscales so a 7-point tensor Gauss rule
    # of the 6-D integrand is accurate to ~1e-10
    p.edges = [np.linspace(0.0, 0.2, 3), np.linspace(0.1, 0.3, 3), np.linspace(0.0, 0.16, 3)]
    p.lengthscale = (0.15, 0.2, 0.18)
    o = O.Oracle(p)
    G = o.volume_gram()
    cells = _cells(p)
    cc = p.cell_coef
    for (i, j) in [(0, 0), (1, 6), (3, 4)]:
        ref = _brute_volume_pair(cells[i], cells[j], p.lengthscale, _terms(p), n=7, cc=(cc[i], cc[j]))
        assert abs(G[i, j] - ref) <= 1e-8 * max(1.0, abs(ref)), (i, j, G[i, j], ref)


def test_cross_and_grid_covariances_bruteforce():
    p = _small_heat()
    o = O.Oracle(p)
    Gbp = o.cross_gram()
    cells = _cells(p)
    pts = []
    for g in p.groups:
        mesh = np.meshgrid(*g.axes, indexing="ij")
        pts += [tuple(m.ravel()[k] for m in mesh) for k in range(g.size)]
    terms = _terms(p)
    for (b, v) in [(0, 0), (2, 3), (5, 5), (7, 1)]:
        X2, w2 = _box_rule(cells[v], 10)
        A = np.tile(np.array(pts[b]), (len(X2), 1))
        vals = _apply_op(lambda x, y: _kernel(x, y, p.lengthscale), torch.from_numpy(A),
                         torch.from_numpy(X2), [((0, 0), 1.0)], [(a, c) for (a, c, _) in terms]).numpy()
        ref = float((vals * w2).sum())
        assert abs(Gbp[b, v] - ref) <= 1e-11 * max(1.0, abs(ref))
    # L_V k(x) at evaluation points (first argument integrated)
    X = np.array([[0.3, 0.45], [0.9, 0.05]])
    kb, kp = o.Lk_points(X)
    for m in range(2):
        for v in (0, 4):
            X1, w1 = _box_rule(cells[v], 10)
            A = np.tile(X[m], (len(X1), 1))
            vals = _apply_op(lambda x, y: _kernel(x, y, p.lengthscale), torch.from_numpy(X1),
                             torch.from_numpy(A), [(a, c) for (a, c, _) in terms], [((0, 0), 1.0)]).numpy()
            ref = float((vals * w1).sum())
            assert abs(kp[v, m] - ref) <= 1e-11 * max(1.0, abs(ref))
        for b in (0, 5):
            ref = float(_kernel(torch.tensor([pts[b]]), torch.tensor([X[m]]), p.lengthscale)[0])
            assert abs(kb[b, m] - ref) < 1e-14


def test_derivative_point_observation_bruteforce():
    """u_t point observations (wave IC velocity) against autograd."""
    p = W.wave2d_c4(nt=2, nx=2, ny=2, n_ic=2, n_bt=2, n_bs=1, grid_t=2)
    o = O.Oracle(p)
    Gbb = o.point_gram()
    g0, g1 = p.groups[0], p.groups[1]
    pts0 = np.stack([m.ravel() for m in np.meshgrid(*g0.axes, indexing="ij")], 1)
    pts1 = np.stack([m.ravel() for m in np.meshgrid(*g1.axes, indexing="ij")], 1)
    f = lambda x, y: _kernel(x, y, p.lengthscale)
    ref = _apply_op(f, torch.from_numpy(pts0[[1]]), torch.from_numpy(pts1[[2]]),
                    [((0, 0, 0), 1.0)], [((1, 0, 0), 1.0)]).numpy()[0]
    assert abs(Gbb[1, g0.size + 2] - ref) < 1e-14
    ref = _apply_op(f, torch.from_numpy(pts1[[0]]), torch.from_numpy(pts1[[3]]),
                    [((1, 0, 0), 1.0)], [((1, 0, 0), 1.0)]).numpy()[0]
    assert abs(Gbb[g0.size, g0.size + 3] - ref) < 1e-12


@pytest.mark.parametrize("mk", [lambda: W.heat1d_c1(nt=6, nx=5, n_ic=8),
                                lambda: W.advdiff_c2(nt=5, nx=6, n_ic=8),
                                lambda: W.wave2d_c4(nt=3, nx=4, ny=3, n_ic=3, n_bt=2, n_bs=2)])
def test_gram_symmetric_psd_and_matrix_free_consistent(mk):
    p = mk()
    o = O.Oracle(p)
    G = o.gram()
    assert np.abs(G - G.T).max() <= 1e-14 * np.abs(G).max()
    ev = np.linalg.eigvalsh(G)
    assert ev.min() >= -1e-12 * ev.max()
    rng = np.random.default_rng(0)
    v = rng.standard_normal(p.n_pde)
    assert np.allclose(o.volume_matvec(v), o.volume_gram() @ v, rtol=1e-12, atol=1e-14 * np.abs(G).max())
    Gbp = o.cross_gram()
    assert np.allclose(o.cross_matvec(v), Gbp @ v, rtol=1e-12, atol=1e-15)
    w = rng.standard_normal(p.n_b)
    assert np.allclose(o.cross_rmatvec(w), Gbp.T @ w, rtol=1e-12, atol=1e-15)
    assert np.allclose(o.volume_diag(), np.diag(o.volume_gram()), rtol=1e-13)
