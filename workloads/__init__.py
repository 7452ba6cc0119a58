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
    "PointGroup", "PDETerm", "IBVP", "uniform_edges", "centres",
    "heat1d_c1", "advdiff_c2", "heat2d_c3", "wave2d_c4", "serving_trace",
    "heat2d_request", "scaled", "CONFIGS", "wave2d_benchmark", "wave2d_benchmark_solution",
]


@dataclass
class PointGroup:
    """A tensor grid of point observations ``d^beta u(x) = y + eps``."""
    axes: List[np.ndarray]            # one coordinate array per dim (len 1 pins it)
    deriv: Tuple[int, ...]            # derivative multi-index beta
    y: np.ndarray                     # prod(len(axes[i])) values, row-major
    noise_var: float                  # variance of eps (absolute)

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(len(a) for a in self.axes)

    @property
    def size(self) -> int:
        return int(np.prod(self.shape))


@dataclass
class PDETerm:
    """One summand ``coef * d^alpha u`` of the operator D (optionally times a
    per-cell coefficient, paper Appendix 'Variable bathymetry')."""
    alpha: Tuple[int, ...]
    coef: float
    cellwise: bool = False


@dataclass
class IBVP:
    name: str
    d: int
    edges: List[np.ndarray]                  # per dim, N_i + 1 increasing values
    lengthscale: Tuple[float, ...]
    outputscale: float                       # sigma_f^2
    terms: List[PDETerm]
    groups: List[PointGroup]
    cell_coef: Optional[np.ndarray] = None   # N values (per-volume coefficient)
    f_int: Optional[np.ndarray] = None       # N values of the integral of f over V; None = 0
    noise_pde: float = 1e-6                  # PDE-observation noise
    noise_pde_relative: bool = True          # True: variance = noise_pde * mean diag of the volume Gram
    grid: List[np.ndarray] = field(default_factory=list)   # posterior grid axes
    meta: dict = field(default_factory=dict)
    # per-dimension kernel: 0 = squared exponential, 1..4 = Matern nu = 1/2, 3/2, 5/2, 7/2
    kernel: Tuple[int, ...] = ()

    def kernel_codes(self) -> Tuple[int, ...]:
        return tuple(self.kernel[i] if i < len(self.kernel) else 0 for i in range(self.d))

    @property
    def ncell(self) -> Tuple[int, ...]:
        return tuple(len(e) - 1 for e in self.edges)

    @property
    def n_pde(self) -> int:
        return int(np.prod(self.ncell))

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
}
