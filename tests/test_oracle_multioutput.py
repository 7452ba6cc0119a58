"""Pins of the oracle's multi-output path (Sec. 3.3 eq. multioutput-cov-def:
independent outputs; the linearised shallow-water system of the appendix
"Tsunami propagation", eq. sw1 to sw3, with a radiation boundary condition).

  - a system whose equations and point groups each touch one output is two
    separate single-output problems (Gram and posterior);
  - equations and point observations on u0 + u1 and u0 - u1 of two iid outputs
    are two independent single-output problems on w+- = u0 +- u1 (prior 2k),
    so the coupled Gram is block diagonal and u0 = (w+ + w-)/2;
  - Gram entries of a small shallow-water system (per-cell H, Coriolis, drag,
    two-term radiation rows with per-point wave speeds) against brute-force
    quadrature of the operators applied by automatic differentiation;
  - the posterior mean of a Poincare plane wave (an exact solution of sw1 to
    sw3 at constant depth) converges to it, and a sign slip in the Coriolis
    terms breaks that."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as W
from oracle import gpfvm_oracle as O


def _pair_system(nt=3, nx=4, seed=11):
    """Heat on u0 (equation 0) and advection-diffusion on u1 (equation 1),
    each with its own initial values; shared grid and kernel."""
    rng = np.random.default_rng(seed)
    edges = [W.uniform_edges(0, 1, nt), W.uniform_edges(0, 1, nx)]
    ta = [W.PDETerm((1, 0), 1.0), W.PDETerm((0, 2), -0.1)]
    tb = [W.PDETerm((1, 0), 1.0), W.PDETerm((0, 1), 0.5), W.PDETerm((0, 2), -0.01)]
    xa, xb = W.centres(5), W.centres(6)
    ga = [W.PointGroup([np.array([0.0]), xa], (0, 0), np.sin(np.pi * xa), 1e-6),
          W.PointGroup([W.centres(nt), np.array([0.0])], (0, 0), np.zeros(nt), 1e-6)]
    gb = [W.PointGroup([np.array([0.0]), xb], (0, 0), np.cos(2 * xb), 1e-6)]
    fa, fb = rng.normal(0, 0.1, nt * nx), rng.normal(0, 0.1, nt * nx)
    common = dict(d=2, edges=edges, lengthscale=(0.3, 0.25), noise_pde=1e-4, noise_pde_relative=False,
                  grid=[W.centres(3), W.centres(5)], kernel=(3, 3))
    A = W.IBVP(name="a", outputscale=1.0, terms=ta, groups=ga, f_int=fa, **common)
    B = W.IBVP(name="b", outputscale=2.5, terms=tb, groups=gb, f_int=fb, **common)
    mt = [dataclasses.replace(t, out=0, eq=0) for t in ta] + [dataclasses.replace(t, out=1, eq=1) for t in tb]
    mg = [dataclasses.replace(g, out=0) for g in ga] + [dataclasses.replace(g, out=1) for g in gb]
    AB = W.IBVP(name="ab", outputscale=1.0, terms=mt, groups=mg, f_int=np.concatenate([fa, fb]), nout=2, neq=2,
                out_scale=(1.0, 2.5), **common)
    return A, B, AB


def test_decoupled_system_is_two_single_output_problems():
    A, B, AB = _pair_system()
    oa, ob, om = O.Oracle(A), O.Oracle(B), O.Oracle(AB)
    # observation order of the system: [points of A; points of B; volumes of A; volumes of B]
    ia = np.r_[0:A.n_b, A.n_b + B.n_b + np.arange(A.n_pde)]
    ib = np.r_[A.n_b:A.n_b + B.n_b, A.n_b + B.n_b + A.n_pde + np.arange(B.n_pde)]
    G = om.gram()
    assert np.allclose(G[np.ix_(ia, ia)], oa.gram(), rtol=0, atol=1e-13)
    assert np.allclose(G[np.ix_(ib, ib)], ob.gram(), rtol=0, atol=1e-13)
    assert np.abs(G[np.ix_(ia, ib)]).max() == 0.0
    X = om.grid_points(A.grid)
    for out, (o, p) in enumerate(((oa, A), (ob, B))):
        m, v, _ = O.dense_posterior(om, X, out=out)
        m1, v1, _ = O.dense_posterior(o, X)
        assert np.allclose(m, m1, rtol=0, atol=1e-9 * max(1.0, np.abs(m1).max()))
        assert np.allclose(v, v1, rtol=0, atol=1e-9 * p.outputscale)


def _rotated(seed=12, nt=3, nx=4):
    """Single problem P (heat, prior 2k) and the coupled system on (u0, u1)
    whose observations are those of P on w+ = u0 + u1 and on w- = u0 - u1."""
    rng = np.random.default_rng(seed)
    edges = [W.uniform_edges(0, 1, nt), W.uniform_edges(0, 1, nx)]
    terms = [W.PDETerm((1, 0), 1.0), W.PDETerm((0, 2), -0.1), W.PDETerm((0, 1), 0.3)]
    xi = W.centres(5)
    yp, ym = np.sin(np.pi * xi), 0.5 * np.cos(np.pi * xi)
    fp, fm = rng.normal(0, 0.1, nt * nx), rng.normal(0, 0.1, nt * nx)
    common = dict(d=2, edges=edges, lengthscale=(0.3, 0.25), noise_pde=1e-4, noise_pde_relative=False,
                  grid=[W.centres(3), W.centres(5)], kernel=(0, 0))
    ic = lambda y: W.PointGroup([np.array([0.0]), xi], (0, 0), y, 1e-6)
    Pp = W.IBVP(name="p", outputscale=2.0, terms=terms, groups=[ic(yp)], f_int=fp, **common)
    Pm = W.IBVP(name="m", outputscale=2.0, terms=terms, groups=[ic(ym)], f_int=fm, **common)
    mt = []
    for eq, sgn in ((0, 1.0), (1, -1.0)):
        for t in terms:
            mt += [dataclasses.replace(t, out=0, eq=eq), dataclasses.replace(t, coef=sgn * t.coef, out=1, eq=eq)]
    mg = [W.PointGroup([np.array([0.0]), xi], (0, 0), y, 1e-6,
                       terms=[W.PointTerm((0, 0), 1.0, 0), W.PointTerm((0, 0), sgn, 1)])
          for y, sgn in ((yp, 1.0), (ym, -1.0))]
    S = W.IBVP(name="rot", outputscale=1.0, terms=mt, groups=mg, f_int=np.concatenate([fp, fm]), nout=2, neq=2,
               **common)
    return Pp, Pm, S


def test_rotated_outputs_are_sum_and_difference_problems():
    Pp, Pm, S = _rotated()
    op, om_, os_ = O.Oracle(Pp), O.Oracle(Pm), O.Oracle(S)
    nb, N = Pp.n_b, Pp.n_pde
    ip = np.r_[0:nb, 2 * nb + np.arange(N)]
    im = np.r_[nb:2 * nb, 2 * nb + N + np.arange(N)]
    G = os_.gram()
    Gp = op.gram()
    assert np.allclose(G[np.ix_(ip, ip)], Gp, rtol=0, atol=1e-13 * np.abs(Gp).max())
    assert np.allclose(G[np.ix_(im, im)], Gp, rtol=0, atol=1e-13 * np.abs(Gp).max())
    assert np.abs(G[np.ix_(ip, im)]).max() <= 1e-13 * np.abs(Gp).max()
    X = os_.grid_points(Pp.grid)
    mp, vp, _ = O.dense_posterior(op, X)
    mm, vm, _ = O.dense_posterior(om_, X)
    for out, sgn in ((0, 1.0), (1, -1.0)):
        m, v, _ = O.dense_posterior(os_, X, out=out)
        assert np.allclose(m, 0.5 * (mp + sgn * mm), rtol=0, atol=1e-9)
        assert np.allclose(v, 0.25 * (vp + vm), rtol=0, atol=1e-9)


# ---- brute force on a small shallow-water system ------------------------------

def _kernel(x, x2, ell):
    z = ((x - x2) / torch.tensor(ell, dtype=torch.float64)) ** 2
    return torch.exp(-0.5 * z.sum(dim=1))


def _apply(x, x2, ell, terms1, terms2):
    """sum c1 c2 d^a1_x d^a2_x2 k at every row (autograd)."""
    out = torch.zeros(x.shape[0], dtype=torch.float64)
    for (a1, c1) in terms1:
        for (a2, c2) in terms2:
            xx = x.clone().requires_grad_(True)
            yy = x2.clone().requires_grad_(True)
            val = _kernel(xx, yy, ell)
            for dim, order in enumerate(a1):
                for _ in range(order):
                    val = torch.autograd.grad(val.sum(), xx, create_graph=True)[0][:, dim]
            for dim, order in enumerate(a2):
                for _ in range(order):
                    val = torch.autograd.grad(val.sum(), yy, create_graph=True)[0][:, dim]
            out = out + c1 * c2 * val.detach()
    return out


def _box(box, n):
    rules = [np.polynomial.legendre.leggauss(n) for _ in box]
    pts = [0.5 * (b - a) * x + 0.5 * (a + b) for (a, b), (x, _) in zip(box, rules)]
    wts = [0.5 * (b - a) * w for (a, b), (_, w) in zip(box, rules)]
    X = np.stack([m.ravel() for m in np.meshgrid(*pts, indexing="ij")], 1)
    w = np.prod(np.stack([m.ravel() for m in np.meshgrid(*wts, indexing="ij")], 1), axis=1)
    return X, w


def _small_sw():
    p = W.shallow_water(nt=2, nx=2, ny=2, n_icx=2, n_icy=2, n_bt=2, n_bx=2, n_by=2, kernel=0,
                        lengthscale=(0.15, 0.2, 0.18), f_cor=0.7, drag=0.3, out_scale=(1.0, 1.7, 0.6))
    # narrow cells against the lengthscales: a 7-point Gauss rule per dimension is accurate to ~1e-10
    p.edges = [np.linspace(0.0, 0.2, 3), np.linspace(0.1, 0.3, 3), np.linspace(0.0, 0.16, 3)]
    return p


def _obs_terms(p, row):
    """Observation `row` as (kind, data, {out: [(alpha, coef)]})."""
    if row < p.n_b:
        off = 0
        for g in p.groups:
            if row < off + g.size:
                k = row - off
                idx = np.unravel_index(k, g.shape)
                x = np.array([g.axes[i][idx[i]] for i in range(p.d)])
                per = {}
                for c in g.components():
                    w = c.weight_grid(g.shape)[k]
                    per.setdefault(c.out, []).append((c.deriv, c.coef * w))
                return "point", x, per
            off += g.size
    v = row - p.n_b
    eq, cell = divmod(v, p.n_cells)
    idx = np.unravel_index(cell, p.ncell)
    box = [(p.edges[i][idx[i]], p.edges[i][idx[i] + 1]) for i in range(p.d)]
    per = {}
    for t in p.terms:
        if t.eq == eq:
            per.setdefault(t.out, []).append((t.alpha, t.coef * (p.cell_coef[cell] if t.cellwise else 1.0)))
    return "cell", box, per


def _brute(p, r1, r2, n=7):
    k1, d1, t1 = _obs_terms(p, r1)
    k2, d2, t2 = _obs_terms(p, r2)
    X1, w1 = (d1[None, :], np.ones(1)) if k1 == "point" else _box(d1, n)
    X2, w2 = (d2[None, :], np.ones(1)) if k2 == "point" else _box(d2, n)
    A = torch.from_numpy(np.repeat(X1, len(X2), 0)); B = torch.from_numpy(np.tile(X2, (len(X1), 1)))
    wt = np.repeat(w1, len(w2)) * np.tile(w2, len(w1))
    total = 0.0
    for out, sf in enumerate(p.output_scales()):
        if out in t1 and out in t2:
            total += sf * float((_apply(A, B, p.lengthscale, t1[out], t2[out]).numpy() * wt).sum())
    return total


def test_shallow_water_gram_matches_bruteforce():
    p = _small_sw()
    o = O.Oracle(p)
    G = o.gram()
    nb, Nc = p.n_b, p.n_cells
    G[nb:, nb:] -= o.noise_pde() * np.eye(p.n_pde)
    G[:nb, :nb] -= np.diag(np.concatenate([np.full(g.size, g.noise_var) for g in p.groups]))
    gs = np.cumsum([0] + [g.size for g in p.groups])
    rad_x, rad_y = gs[3], gs[5]                 # first rows of an x-edge and a y-edge radiation group
    pairs = [(nb + 1, nb + 1), (nb + 0, nb + Nc + 3), (nb + Nc + 2, nb + 2 * Nc + 5), (nb + 2 * Nc + 7, nb + 2 * Nc + 1),
             (nb + 4, nb + 2 * Nc + 6),
             (rad_x, rad_x), (rad_x + 1, rad_y + 2), (rad_y + 3, gs[6]), (0, rad_x + 2), (gs[1], gs[2]),
             (rad_x, nb + 5), (rad_y + 1, nb + Nc + 2), (gs[1] + 1, nb + 2 * Nc + 4), (0, nb + Nc + 6)]
    for r1, r2 in pairs:
        ref = _brute(p, r1, r2)
        assert abs(G[r1, r2] - ref) <= 1e-8 * max(1.0, abs(ref)), (r1, r2, G[r1, r2], ref)
        assert abs(G[r2, r1] - ref) <= 1e-8 * max(1.0, abs(ref)), (r2, r1, G[r2, r1], ref)
    assert G[0, gs[1]] == 0.0 and G[gs[1], gs[2]] == 0.0     # initial values of different outputs


# ---- Poincare plane wave --------------------------------------------------------

def _plane_wave(nt, nx, f_cor, flip=False, g=1.0, kx=2 * np.pi, A=1.0):
    """h = A cos(kx x - w t), u = (A w / kx) cos(.), v = (f A / kx) sin(.),
    w^2 = f^2 + g kx^2 (H = 1, no drag): an exact solution of sw1 to sw3 that
    does not depend on y.  Initial values of (h, u, v) and boundary values of
    h at x = 0 and x = 1, observed at y = 1/2; one cell in y."""
    w = np.sqrt(f_cor ** 2 + g * kx ** 2)
    exact = lambda t, x: (A * np.cos(kx * x - w * t), A * w / kx * np.cos(kx * x - w * t),
                          f_cor * A / kx * np.sin(kx * x - w * t))
    xi, tb, mid = W.centres(2 * nx), W.centres(2 * nt), np.array([0.5])
    h0, u0, v0 = exact(0.0, xi)
    groups = [W.PointGroup([np.array([0.0]), xi, mid], (0, 0, 0), y, 1e-10, out=o)
              for o, y in enumerate((h0, u0, v0))]
    for xe in (0.0, 1.0):
        groups.append(W.PointGroup([tb, np.array([xe]), mid], (0, 0, 0), exact(tb, xe)[0], 1e-10, out=0))
    terms = W.sw_terms(g, -f_cor if flip else f_cor, 0.0, H_cellwise=False)
    p = W.IBVP(name="plane", d=3, edges=[W.uniform_edges(0, 0.5, nt), W.uniform_edges(0, 1, nx),
                                         W.uniform_edges(0, 1, 1)],
               lengthscale=(0.15, 0.15, 3.0), outputscale=1.0, terms=terms, groups=groups, noise_pde=1e-10,
               noise_pde_relative=False, kernel=(0, 0, 0), nout=3, neq=3, out_scale=(1.0, 1.5, 0.3))
    T, X = np.meshgrid(np.linspace(0.05, 0.45, 5), np.linspace(0.05, 0.95, 7), indexing="ij")
    pts = np.stack([T.ravel(), X.ravel(), np.full(T.size, 0.5)], 1)
    return p, pts, exact(T.ravel(), X.ravel())


def _wave_errors(nt, nx, f_cor, flip=False):
    """max |mean - exact| per output (h, u, v), relative to h's amplitude 1."""
    p, X, ex = _plane_wave(nt, nx, f_cor, flip)
    o = O.Oracle(p)
    return [float(np.abs(O.dense_posterior(o, X, out=out)[0] - ex[out]).max()) for out in range(3)]


def test_plane_wave_posterior_converges_and_a_coriolis_sign_slip_breaks_it():
    coarse = _wave_errors(4, 8, 3.0)
    fine = _wave_errors(8, 16, 3.0)
    slip = _wave_errors(8, 16, 3.0, flip=True)
    # h (observed on both x-edges) converges with the cells; u and v, fixed by
    # their initial values and the three equations, stay within 3e-2
    assert max(fine) < 3e-2 and fine[0] < 0.5 * coarse[0], (coarse, fine)
    assert min(slip) > 10 * max(fine), (fine, slip)
