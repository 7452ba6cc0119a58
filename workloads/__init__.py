"""Seeded synthetic IBVP workloads shared by the CPU oracle and the HIP path.

This module only *describes* problems: domains, cell edges, the PDE operator
as a list of (derivative multi-index, coefficient) pairs, point-observation
groups with their data, and evaluation grids.  It holds none of the GP-FVM
arithmetic (no kernel derivatives, no cell integrals, no Gram, no solver), so
the oracle and the library can both consume it without sharing method code.

Problem class (paper, Sec. 1 eq. def-lin-pde and Sec. 2.2): a linear PDE
``D[u] = f`` on ``[0,T] x X`` with initial/boundary point observations,
discretised by box volumes with factorised structure (Sec. 4.1, Definition of
a box FVM scheme).  Dimension 0 is time.  Volumes are flattened row-major with
time slowest; every point group is a tensor grid flattened the same way.

The random draws used to build data (GP-drawn initial conditions, bump
centres, bathymetry) use ``numpy.random.default_rng(seed)``.  The GP draws
sample a separable squared-exponential field on a tensor grid by factorising
each 1-D covariance separately (sample = L_0 Z L_1^T); that is data synthesis,
not part of the method.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "PointTerm", "PointGroup", "PDETerm", "IBVP", "uniform_edges", "centres",
    "heat1d_c1", "advdiff_c2", "heat2d_c3", "wave2d_c4", "serving_trace",
    "heat2d_request", "scaled", "CONFIGS", "wave2d_benchmark", "wave2d_benchmark_solution",
    "shallow_water", "sw_depth", "sw_terms",
]


@dataclass
class PointTerm:
    """One summand ``coef * w(x) * d^beta u_out(x)`` of a point observation.
    The per-point weight is separable: w(x) = prod_i weights[i][j_i] over the
    group's grid indices (None: 1 in that dimension), e.g. the wave speed of a
    radiation boundary condition along its edge."""
    deriv: Tuple[int, ...]
    coef: float = 1.0
    out: int = 0
    weights: Optional[List[Optional[np.ndarray]]] = None

    def weight_grid(self, shape: Sequence[int]) -> np.ndarray:
        """w over the group's points, row-major (prod(shape) values)."""
        w = np.ones(tuple(shape))
        for i, n in enumerate(shape):
            if self.weights is not None and self.weights[i] is not None:
                wi = np.asarray(self.weights[i], float)
                assert wi.shape == (n,)
                w = w * wi.reshape([n if k == i else 1 for k in range(len(shape))])
        return w.ravel()


@dataclass
class PointGroup:
    """A tensor grid of point observations ``d^beta u_out(x) = y + eps``, or,
    with ``terms``, of a sum of such terms (e.g. h_t - c h_x = 0)."""
    axes: List[np.ndarray]            # one coordinate array per dim (len 1 pins it)
    deriv: Tuple[int, ...]            # derivative multi-index beta (single-term form)
    y: np.ndarray                     # prod(len(axes[i])) values, row-major
    noise_var: float                  # variance of eps (absolute)
    out: int = 0                      # observed output (single-term form)
    terms: Optional[List[PointTerm]] = None   # multi-term form (replaces deriv/out)

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(len(a) for a in self.axes)

    @property
    def size(self) -> int:
        return int(np.prod(self.shape))

    def components(self) -> List[PointTerm]:
        if self.terms:
            return list(self.terms)
        return [PointTerm(tuple(self.deriv), 1.0, self.out, None)]


@dataclass
class PDETerm:
    """One summand ``coef * d^alpha u_out`` of equation ``eq`` of the operator
    (optionally times a per-cell coefficient, paper Appendix 'Variable
    bathymetry').  Several equations over several outputs form a system such
    as the linearised shallow-water equations (Sec. 3.3)."""
    alpha: Tuple[int, ...]
    coef: float
    cellwise: bool = False
    out: int = 0
    eq: int = 0


@dataclass
class IBVP:
    name: str
    d: int
    edges: List[np.ndarray]                  # per dim, N_i + 1 increasing values
    lengthscale: Tuple[float, ...]
    outputscale: float                       # sigma_f^2
    terms: List[PDETerm]
    groups: List[PointGroup]
    cell_coef: Optional[np.ndarray] = None   # one value per cell (per-volume coefficient)
    f_int: Optional[np.ndarray] = None       # neq x cells values of the integral of f over V; None = 0
    noise_pde: float = 1e-6                  # PDE-observation noise
    noise_pde_relative: bool = True          # True: variance = noise_pde * mean diag of the volume Gram
    grid: List[np.ndarray] = field(default_factory=list)   # posterior grid axes
    meta: dict = field(default_factory=dict)
    # per-dimension kernel: 0 = squared exponential, 1..4 = Matern nu = 1/2, 3/2, 5/2, 7/2
    kernel: Tuple[int, ...] = ()
    # multi-output prior (Sec. 3.3 eq. multioutput-cov-def): nout independent
    # outputs with the same tensor-product kernel and their own outputscales,
    # neq equations observed on every cell (observation order: equation-major)
    nout: int = 1
    neq: int = 1
    out_scale: Optional[Tuple[float, ...]] = None   # sigma_i^2 per output; None: outputscale

    def kernel_codes(self) -> Tuple[int, ...]:
        return tuple(self.kernel[i] if i < len(self.kernel) else 0 for i in range(self.d))

    def output_scales(self) -> Tuple[float, ...]:
        if self.out_scale is None:
            return tuple(float(self.outputscale) for _ in range(self.nout))
        assert len(self.out_scale) == self.nout
        return tuple(float(v) for v in self.out_scale)

    @property
    def ncell(self) -> Tuple[int, ...]:
        return tuple(len(e) - 1 for e in self.edges)

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.ncell))

    @property
    def n_pde(self) -> int:
        """Volume observations: one per equation and cell."""
        return self.neq * self.n_cells

    @property
    def n_b(self) -> int:
        return sum(g.size for g in self.groups)

    @property
    def n(self) -> int:
        return self.n_b + self.n_pde

    def y_obs(self) -> np.ndarray:
        """Observation vector in observation order [points; volumes]."""
        yb = [g.y.ravel() for g in self.groups]
        yp = np.zeros(self.n_pde) if self.f_int is None else np.asarray(self.f_int, float).ravel()
        return np.concatenate(yb + [yp])


def uniform_edges(lo: float, hi: float, n: int) -> np.ndarray:
    return np.linspace(lo, hi, n + 1)


def centres(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Midpoints (j + 1/2)/n of n equal sub-intervals of [lo, hi]."""
    return lo + (hi - lo) * (np.arange(n) + 0.5) / n


def _se_chol(x: np.ndarray, ell: float, jitter: float) -> np.ndarray:
    c = np.exp(-0.5 * ((x[:, None] - x[None, :]) / ell) ** 2) + jitter * np.eye(len(x))
    return np.linalg.cholesky(c)


def gp_draw_grid(axes: Sequence[np.ndarray], ell: float, rng, jitter: float = 1e-10) -> np.ndarray:
    """One draw of a zero-mean unit-variance separable SE field on a tensor
    grid (data synthesis for initial conditions and bathymetry)."""
    z = rng.standard_normal(tuple(len(a) for a in axes))
    for i, a in enumerate(axes):
        L = _se_chol(np.asarray(a, float), ell, jitter)
        z = np.moveaxis(np.tensordot(L, np.moveaxis(z, i, 0), axes=(1, 0)), 0, i)
    return z


# --------------------------------------------------------------------------
# The five workloads.  Readings of the paper's silent points are recorded in
# ``meta['readings']`` so a test or bench line can print them.
# --------------------------------------------------------------------------

NOISE_EXACT = 1e-8     # variance for noise-free point observations
TAU_PDE = 1e-6         # PDE noise variance relative to the mean volume-Gram diagonal


def heat1d_c1(nt: int = 16, nx: int = 16, seed: int = 1, n_ic: int = 32, grid_n: int = 64) -> IBVP:
    """u_t = 0.1 u_xx on [0,1]x[0,1]; IC sin(pi x) + N(0,1e-3); Dirichlet 0."""
    rng = np.random.default_rng(seed)
    xi = centres(n_ic)
    y0 = np.sin(np.pi * xi) + rng.normal(0.0, np.sqrt(1e-3), n_ic)
    tb = centres(nt)
    groups = [
        PointGroup([np.array([0.0]), xi], (0, 0), y0, 1e-3),
        PointGroup([tb, np.array([0.0])], (0, 0), np.zeros(nt), NOISE_EXACT),
        PointGroup([tb, np.array([1.0])], (0, 0), np.zeros(nt), NOISE_EXACT),
    ]
    g = np.linspace(0.0, 1.0, grid_n)
    return IBVP(
        name=f"heat1d_{nt}x{nx}", d=2,
        edges=[uniform_edges(0, 1, nt), uniform_edges(0, 1, nx)],
        lengthscale=(0.2, 0.3), outputscale=1.0,
        terms=[PDETerm((1, 0), 1.0), PDETerm((0, 2), -0.1)],
        groups=groups, noise_pde=TAU_PDE, grid=[g, g.copy()],
        meta={"kappa": 0.1, "analytic": "exp(-0.1 pi^2 t) sin(pi x)"},
    )


def advdiff_c2(nt: int = 128, nx: int = 128, seed: int = 2, n_ic: int = 256) -> IBVP:
    """u_t + 0.5 u_x = 0.01 u_xx on [0,1]^2; IC = seeded SE-GP draw (l=0.1)."""
    rng = np.random.default_rng(seed)
    xi = centres(n_ic)
    y0 = gp_draw_grid([xi], 0.1, rng)
    groups = [PointGroup([np.array([0.0]), xi], (0, 0), y0.ravel(), NOISE_EXACT)]
    return IBVP(
        name=f"advdiff_{nt}x{nx}", d=2,
        edges=[uniform_edges(0, 1, nt), uniform_edges(0, 1, nx)],
        lengthscale=(0.2, 0.1), outputscale=1.0,
        terms=[PDETerm((1, 0), 1.0), PDETerm((0, 1), 0.5), PDETerm((0, 2), -0.01)],
        groups=groups, noise_pde=TAU_PDE, grid=[centres(nt), centres(nx)],
        meta={"beta": 0.5, "nu": 0.01},
    )


def _edge_groups_2d(tb: np.ndarray, sb: np.ndarray) -> List[PointGroup]:
    """Dirichlet-0 observations on the four spatial edges of [0,1]^2."""
    z = np.zeros(len(tb) * len(sb))
    zero, one = np.array([0.0]), np.array([1.0])
    return [
        PointGroup([tb, zero, sb], (0, 0, 0), z.copy(), NOISE_EXACT),
        PointGroup([tb, one, sb], (0, 0, 0), z.copy(), NOISE_EXACT),
        PointGroup([tb, sb, zero], (0, 0, 0), z.copy(), NOISE_EXACT),
        PointGroup([tb, sb, one], (0, 0, 0), z.copy(), NOISE_EXACT),
    ]


def heat2d_c3(nt: int = 64, nx: int = 64, ny: int = 64, seed: int = 3, n_ic: int = 64,
              n_bt: int = 64, n_bs: int = 32, kappa: float = 0.01, grid_t: int = 16) -> IBVP:
    """u_t = kappa (u_xx + u_yy) on [0,1]^3; IC = 4 seeded Gaussian bumps."""
    rng = np.random.default_rng(seed)
    ctr = rng.uniform(0.2, 0.8, size=(4, 2))
    wid = rng.uniform(0.05, 0.15, size=4)
    xi = centres(n_ic)
    X, Y = np.meshgrid(xi, xi, indexing="ij")
    u0 = sum(np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2 * w * w)) for c, w in zip(ctr, wid))
    groups = [PointGroup([np.array([0.0]), xi, xi.copy()], (0, 0, 0), u0.ravel(), NOISE_EXACT)]
    groups += _edge_groups_2d(centres(n_bt), centres(n_bs))
    return IBVP(
        name=f"heat2d_{nt}x{nx}x{ny}", d=3,
        edges=[uniform_edges(0, 1, nt), uniform_edges(0, 1, nx), uniform_edges(0, 1, ny)],
        lengthscale=(0.2, 0.1, 0.1), outputscale=1.0,
        terms=[PDETerm((1, 0, 0), 1.0), PDETerm((0, 2, 0), -kappa), PDETerm((0, 0, 2), -kappa)],
        groups=groups, noise_pde=TAU_PDE, grid=[centres(grid_t), centres(nx), centres(ny)],
        meta={"kappa": kappa, "bump_centres": ctr.tolist(), "bump_widths": wid.tolist()},
    )


def wave2d_c4(nt: int = 64, nx: int = 128, ny: int = 128, seed: int = 4, n_ic: int = 64,
              n_bt: int = 64, n_bs: int = 32, grid_t: int = 8) -> IBVP:
    """u_tt = div(c^2 grad u) with c^2 = 9.81 H / (9.81 * 200) piecewise constant
    per cell, H a seeded smooth field mapped to [10, 200] m; Gaussian IC."""
    rng = np.random.default_rng(seed)
    xc, yc = centres(nx), centres(ny)
    h = gp_draw_grid([xc, yc], 0.2, rng)
    H = 10.0 + (h - h.min()) / (h.max() - h.min()) * 190.0
    c2 = np.broadcast_to((H / 200.0)[None, :, :], (nt, nx, ny)).ravel().copy()
    xi = centres(n_ic)
    X, Y = np.meshgrid(xi, xi, indexing="ij")
    u0 = np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / (2 * 0.1 ** 2))
    zero = np.array([0.0])
    groups = [
        PointGroup([zero, xi, xi.copy()], (0, 0, 0), u0.ravel(), NOISE_EXACT),
        PointGroup([zero, xi.copy(), xi.copy()], (1, 0, 0), np.zeros(n_ic * n_ic), NOISE_EXACT),
    ]
    groups += _edge_groups_2d(centres(n_bt), centres(n_bs))
    return IBVP(
        name=f"wave2d_{nt}x{nx}x{ny}", d=3,
        edges=[uniform_edges(0, 1, nt), uniform_edges(0, 1, nx), uniform_edges(0, 1, ny)],
        lengthscale=(0.1, 0.1, 0.1), outputscale=1.0,
        terms=[PDETerm((2, 0, 0), 1.0), PDETerm((0, 2, 0), -1.0, True), PDETerm((0, 0, 2), -1.0, True)],
        groups=groups, cell_coef=c2, noise_pde=TAU_PDE,
        grid=[centres(grid_t), xc.copy(), yc.copy()],
        meta={"H_range_m": [10.0, 200.0], "c2_scale": "9.81*H/(9.81*200)"},
    )


def wave2d_benchmark(n: int = 8, seed: int = 0, lengthscale=(0.575, 0.325, 0.325), kernel: int = 3,
                     grid=(8, 16, 16)) -> IBVP:
    """The paper's 2-D wave benchmark (appendix "2D Wave Equation Benchmark"):
    u_tt = c^2 (u_xx + u_yy), c = 1, on [0,2] x [0,1]^2 with n cells per
    dimension; IC sum_{i,j<=2} C_ij sin(i pi x) sin(j pi y) observed on 8 x 8
    uniform points together with u_t(0) = 0 there; Dirichlet 0 on the four
    spatial edges at 20 uniform times x 10 uniform positions each.  C is one
    seeded draw of N((1, .5, .5, 0), diag(.1, .2, .2, .3)^2).  Tensor-product
    Matern kernel (code 3: nu = 5/2) in every dimension.  The exact solution is
    wave2d_benchmark_solution."""
    C = _wave_benchmark_coefs(seed)
    xi = centres(8)
    X, Y = np.meshgrid(xi, xi, indexing="ij")
    u0 = sum(C[i, j] * np.sin((i + 1) * np.pi * X) * np.sin((j + 1) * np.pi * Y) for i in range(2) for j in range(2))
    zero = np.array([0.0])
    groups = [
        PointGroup([zero, xi, xi.copy()], (0, 0, 0), u0.ravel(), NOISE_EXACT),
        PointGroup([zero, xi.copy(), xi.copy()], (1, 0, 0), np.zeros(64), NOISE_EXACT),
    ]
    groups += _edge_groups_2d(centres(20, 0.0, 2.0), centres(10))
    return IBVP(
        name=f"wave2d_benchmark_{n}^3", d=3,
        edges=[uniform_edges(0, 2, n), uniform_edges(0, 1, n), uniform_edges(0, 1, n)],
        lengthscale=tuple(lengthscale), outputscale=1.0,
        terms=[PDETerm((2, 0, 0), 1.0), PDETerm((0, 2, 0), -1.0), PDETerm((0, 0, 2), -1.0)],
        groups=groups, noise_pde=TAU_PDE,
        grid=[centres(grid[0], 0.0, 2.0), centres(grid[1]), centres(grid[2])],
        kernel=(kernel, kernel, kernel),
        meta={"C": C.tolist(), "c": 1.0},
    )


def _wave_benchmark_coefs(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    mean = np.array([1.0, 0.5, 0.5, 0.0])
    std = np.array([0.1, 0.2, 0.2, 0.3])
    return (mean + std * rng.standard_normal(4)).reshape(2, 2)


def wave2d_benchmark_solution(seed: int, axes: Sequence[np.ndarray]) -> np.ndarray:
    """Separation of variables for wave2d_benchmark: each mode sin(i pi x)
    sin(j pi y) oscillates as cos(pi sqrt(i^2 + j^2) t) (c = 1, u_t(0) = 0).
    Values on the tensor grid `axes` (t, x, y), flattened row-major."""
    C = _wave_benchmark_coefs(seed)
    T, X, Y = np.meshgrid(*axes, indexing="ij")
    u = np.zeros(T.shape)
    for i in range(1, 3):
        for j in range(1, 3):
            u += C[i - 1, j - 1] * np.sin(i * np.pi * X) * np.sin(j * np.pi * Y) * np.cos(np.pi * np.hypot(i, j) * T)
    return u.ravel()


def heat2d_request(ns: int, nt: int, seed: int, kappa: float = 0.01, grid_t: int = 8) -> IBVP:
    """One serving request: 2-D heat on [0,1]^3 with nt x ns x ns cells, IC a
    seeded SE-GP draw (l = 0.1) on the ns x ns grid of cell centres,
    Dirichlet 0 on 4 edges x nt x ns/2 points."""
    rng = np.random.default_rng(seed)
    xi = centres(ns)
    u0 = gp_draw_grid([xi, xi], 0.1, rng)
    groups = [PointGroup([np.array([0.0]), xi, xi.copy()], (0, 0, 0), u0.ravel(), NOISE_EXACT)]
    groups += _edge_groups_2d(centres(nt), centres(max(ns // 2, 1)))
    return IBVP(
        name=f"req_{nt}x{ns}x{ns}_s{seed}", d=3,
        edges=[uniform_edges(0, 1, nt), uniform_edges(0, 1, ns), uniform_edges(0, 1, ns)],
        lengthscale=(0.2, 0.1, 0.1), outputscale=1.0,
        terms=[PDETerm((1, 0, 0), 1.0), PDETerm((0, 2, 0), -kappa), PDETerm((0, 0, 2), -kappa)],
        groups=groups, noise_pde=TAU_PDE, grid=[centres(grid_t), xi.copy(), xi.copy()],
        meta={"kappa": kappa},
    )


def sw_depth(x, y, seed: int = 6) -> np.ndarray:
    """Synthetic bathymetry H(x, y) (nondimensional, in [0.05, 1]): an ocean
    of depth 1 rising over a shelf to depth 0.05 at a coast along x = 1; the
    shelf edge x_s(y) and a mild depth modulation follow three seeded Fourier
    modes.  Smooth, so it can be read at cell centres (the per-cell H) and at
    boundary points (the radiation wave speed) alike."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=(3, 3))          # (amplitude, frequency, phase) of 3 modes
    x = np.asarray(x, float); y = np.asarray(y, float)
    xs = 0.72 + sum(0.04 * a[k, 0] * np.sin(2 * np.pi * (k + 1) * y + np.pi * a[k, 2]) for k in range(3))
    shelf = 1.0 / (1.0 + np.exp(-(x - xs) / 0.06))
    mod = 1.0 + sum(0.08 * a[k, 1] * np.cos(2 * np.pi * (k + 1) * (x + y) + np.pi * a[k, 2]) for k in range(3))
    return 0.05 + 0.95 * (1.0 - shelf) * mod


def sw_terms(g: float, f_cor: float, drag: float, H_cellwise: bool = True) -> List[PDETerm]:
    """The three linearised shallow-water equations (eq. sw1 to sw3) as terms
    on the outputs (h, u, v) = (0, 1, 2); H is the per-cell coefficient when
    H_cellwise, else 1 (a constant depth folded into the data's scale)."""
    return [PDETerm((1, 0, 0), 1.0, False, 0, 0), PDETerm((0, 1, 0), 1.0, H_cellwise, 1, 0),
            PDETerm((0, 0, 1), 1.0, H_cellwise, 2, 0),
            PDETerm((1, 0, 0), 1.0, False, 1, 1), PDETerm((0, 0, 0), -f_cor, False, 2, 1),
            PDETerm((0, 1, 0), g, False, 0, 1), PDETerm((0, 0, 0), drag, False, 1, 1),
            PDETerm((1, 0, 0), 1.0, False, 2, 2), PDETerm((0, 0, 0), f_cor, False, 1, 2),
            PDETerm((0, 0, 1), g, False, 0, 2), PDETerm((0, 0, 0), drag, False, 2, 2)]


def shallow_water(nt: int = 20, nx: int = 90, ny: int = 170, seed: int = 6, n_icx: int = 36, n_icy: int = 85,
                  n_bt: int = 40, n_bx: int = 30, n_by: int = 85, g: float = 1.0, f_cor: float = 0.5,
                  drag: float = 0.1, lengthscale=(0.25, 0.06, 0.1), out_scale=(1.0, 2.0, 2.0),
                  grid_t: int = 4, kernel: int = 3) -> IBVP:
    """Linearised 2-D shallow water (appendix "Tsunami propagation", eq. sw1 to
    sw3) on [0,1]^3 in (t, x, y), nondimensional:

        h_t + H (u_x + v_y)      = 0
        u_t - f v + g h_x + k u  = 0
        v_t + f u + g h_y + k v  = 0

    Outputs (h, u, v), each with its own Matern-5/2 tensor-product prior
    (same lengthscales, outputscales ``out_scale``; Sec. 3.3).  H is constant
    per cell (appendix "Variable bathymetry"), the synthetic ``sw_depth`` at
    the cell centre.  The default cell counts are the paper's 20 x 90 x 170
    volumes (three observations each).  Initial condition: an anisotropic
    Gaussian displacement of h (narrow along x), u = v = 0, on an
    n_icx x n_icy grid.  Boundary: the radiation condition h_t = c dh/dn
    pointing inward (h_t - c h_x = 0 at x = 0, h_t + c h_x = 0 at x = 1, the
    same in y), c = sqrt(g H) at the boundary point, on n_bt times x n_by
    (n_bx) points per edge."""
    xc, yc = centres(nx), centres(ny)
    H = sw_depth(xc[:, None], yc[None, :], seed)
    cellH = np.broadcast_to(H[None, :, :], (nt, nx, ny)).ravel().copy()
    xi, yi = centres(n_icx), centres(n_icy)
    X, Y = np.meshgrid(xi, yi, indexing="ij")
    h0 = np.exp(-0.5 * (((X - 0.35) / 0.05) ** 2 + ((Y - 0.5) / 0.15) ** 2))
    zero, one = np.array([0.0]), np.array([1.0])
    groups = [PointGroup([zero, xi, yi.copy()], (0, 0, 0), h0.ravel(), NOISE_EXACT, out=0),
              PointGroup([zero, xi.copy(), yi.copy()], (0, 0, 0), np.zeros(h0.size), NOISE_EXACT, out=1),
              PointGroup([zero, xi.copy(), yi.copy()], (0, 0, 0), np.zeros(h0.size), NOISE_EXACT, out=2)]
    tb, xb, yb = centres(n_bt), centres(n_bx), centres(n_by)
    for edge, sign in ((0.0, -1.0), (1.0, 1.0)):          # x = 0, x = 1: h_t -/+ c h_x = 0
        c = np.sqrt(g * sw_depth(np.full(n_by, edge), yb, seed))
        groups.append(PointGroup([tb.copy(), np.array([edge]), yb.copy()], (1, 0, 0), np.zeros(n_bt * n_by),
                                 NOISE_EXACT, terms=[PointTerm((1, 0, 0), 1.0, 0),
                                                     PointTerm((0, 1, 0), sign, 0, [None, None, c])]))
    for edge, sign in ((0.0, -1.0), (1.0, 1.0)):          # y = 0, y = 1: h_t -/+ c h_y = 0
        c = np.sqrt(g * sw_depth(xb, np.full(n_bx, edge), seed))
        groups.append(PointGroup([tb.copy(), xb.copy(), np.array([edge])], (1, 0, 0), np.zeros(n_bt * n_bx),
                                 NOISE_EXACT, terms=[PointTerm((1, 0, 0), 1.0, 0),
                                                     PointTerm((0, 0, 1), sign, 0, [None, c, None])]))
    terms = sw_terms(g, f_cor, drag)
    return IBVP(
        name=f"shallow_water_{nt}x{nx}x{ny}", d=3,
        edges=[uniform_edges(0, 1, nt), uniform_edges(0, 1, nx), uniform_edges(0, 1, ny)],
        lengthscale=tuple(lengthscale), outputscale=1.0, terms=terms, groups=groups, cell_coef=cellH,
        noise_pde=TAU_PDE, grid=[centres(grid_t), xc.copy(), yc.copy()], kernel=(kernel,) * 3,
        nout=3, neq=3, out_scale=tuple(out_scale),
        meta={"g": g, "f": f_cor, "k": drag, "H_range": [0.05, 1.0], "outputs": ["h", "u", "v"]},
    )


SERVING_NS = (16, 32, 48, 64)
SERVING_NT = (16, 24, 32)


def serving_trace(n_req: int = 512, rate: float = 100.0, seed: int = 5):
    """Poisson arrival trace: list of (arrival_s, ns, nt, request_seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_req)
    arr = np.cumsum(gaps) - gaps[0]
    combos = [(ns, nt) for ns in SERVING_NS for nt in SERVING_NT]
    pick = rng.integers(0, len(combos), size=n_req)
    return [(float(arr[i]), combos[pick[i]][0], combos[pick[i]][1], 5000 + i) for i in range(n_req)]


def scaled(name: str, **kw) -> IBVP:
    """A workload by name, optionally down-scaled (keyword overrides)."""
    return CONFIGS[name](**kw)


CONFIGS = {
    "heat1d": heat1d_c1,
    "advdiff": advdiff_c2,
    "heat2d": heat2d_c3,
    "wave2d": wave2d_c4,
    "shallow_water": shallow_water,
}
