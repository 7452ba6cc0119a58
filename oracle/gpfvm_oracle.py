"""Plain float64 CPU oracle of the GP-FVM hot path (test infrastructure only).

Every function names the passage of the paper it follows.  Notation:
``L`` stacks the observation functionals in the order [IC/BC points; volumes]
(Sec. 2.2, L_IBVP), ``G = L k L' + Sigma`` (Sec. 2.1, Definition and
eq. affine-posterior), volumes are flattened row-major with dimension 0 (time)
slowest.

Parity pins (tests under ``tests/test_oracle_*.py``):
  cell/point factors ......... pinned: closed-form antiderivative forms,
                               mpmath high-precision quadrature, special cases
  Fubini/Kronecker Gram ...... pinned: brute-force tensor Gauss quadrature of
                               the full-dimensional operator (autograd
                               derivatives), symmetry, PSD
  dense posterior ............ pinned: LAPACK Cholesky; noise-free limit
                               interpolates; analytic heat solution convergence
  two-stage Schur solve ...... pinned: equals the one-stage dense solve
  targeted IterGP ............ pinned: with one fixed right-hand side its action
                               residuals are the residuals of textbook CG on
                               that right-hand side; N iterations reproduce the
                               exact posterior; variance non-increasing
  coarse warm start .......... pinned: the aggregated fine Gram equals the
                               coarse scheme's own Gram (subdomain additivity);
                               after the coarse block the posterior equals the
                               exact posterior conditioned on points + coarse
                               volumes; N directions reproduce the exact one
  IterGP ..................... pinned: unit-vector actions reproduce Cholesky;
                               run to n iterations reproduces the exact
                               posterior; combined variance >= exact and
                               non-increasing.  At a fixed k << n (one or two
                               projection passes) the weights and the inverse
                               approximation equal the Galerkin projection onto
                               the Krylov space K_k(S, b), built by Arnoldi on
                               the dense S
  schur_cross ................ pinned: block elimination of the joint Gaussian
                               conditional (full posterior covariance and mean
                               from the dense Gram)
  several outputs ............ pinned: decoupled equations reproduce separate
                               single-output problems; equations on u0 +- u1 of
                               two iid outputs are two problems with prior 2k;
                               shallow-water Gram entries (per-cell H, Coriolis,
                               drag, two-term radiation rows) against brute-force
                               quadrature with autograd derivatives; a Poincare
                               plane wave (exact solution) is recovered
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg as sla

__all__ = [
    "load_quad", "kernel_q", "cell_cell", "point_cell", "point_point", "Oracle",
    "dense_posterior", "itergp", "itergp_targeted", "schur_cross", "cg_solve",
    "coarse_aggregation", "itergp_coarse",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_quad.so")
_lib = None


def build_quad(force: bool = False) -> str:
    """Compile quad.c with gcc (plain C, no GPU)."""
    src = os.path.join(_HERE, "quad.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def load_quad():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_quad())
        d, i, p = ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        for name, args, res in [
            ("ora_kder", [i, d, d], d),
            ("ora_kder_k", [i, i, d, d], d),
            ("ora_point_point", [i, i, i, d, d, d], d),
            ("ora_point_cell", [i, i, i, d, d, d, d], d),
            ("ora_cell_cell", [i, i, i, d, d, d, d, d], d),
            ("ora_integrate_kder", [i, i, d, d, d], d),
            ("ora_qk15_monomial", [i, d, d, p, p], None),
            ("ora_cell_cell_matrix", [i, i, i, i, p, i, p, d, p], None),
            ("ora_point_cell_matrix", [i, i, i, i, p, i, p, d, p], None),
            ("ora_point_point_matrix", [i, i, i, i, p, i, p, d, p], None),
        ]:
            f = getattr(lib, name)
            f.argtypes, f.restype = args, res
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------------------
# 1-D factors (Sec. 3.1 eq. linop-def-univariate; Sec. 3.2 eq. LkL)
# ---------------------------------------------------------------------------

def kernel_q(code: int) -> int:
    """Per-dimension kernel code -> oracle selector: 0 (squared exponential)
    -> -1; 1..4 (Matern nu = 1/2, 3/2, 5/2, 7/2) -> q with nu = q + 1/2."""
    return -1 if code == 0 else code - 1


def _check_order(kq: int, m: int):
    # Matern-(q+1/2) has 2q continuous derivatives; the integrated blocks also
    # accept one order more (a finite jump at r = 0).  Beyond that the
    # pointwise derivative misses a singular part.
    if kq >= 0 and m > 2 * kq + 1:
        raise ValueError(f"derivative order {m} exceeds the smoothness of Matern-{kq}+1/2")


def cell_cell(p: int, q: int, e1: np.ndarray, e2: np.ndarray, ell: float, kq: int = -1) -> np.ndarray:
    """F^{pq}[i, j] = int_{I_i} int_{I'_j} d^p_s d^q_{s'} k(s, s') ds' ds."""
    _check_order(kq, p + q)
    e1 = np.ascontiguousarray(e1, float); e2 = np.ascontiguousarray(e2, float)
    out = np.empty((len(e1) - 1, len(e2) - 1))
    load_quad().ora_cell_cell_matrix(kq, p, q, len(e1) - 1, _ptr(e1), len(e2) - 1, _ptr(e2), ell, _ptr(out))
    return out


def point_cell(p: int, q: int, x: np.ndarray, e2: np.ndarray, ell: float, kq: int = -1) -> np.ndarray:
    """Q^{pq}[i, j] = int_{I'_j} d^p_x d^q_{s'} k(x_i, s') ds'."""
    _check_order(kq, p + q)
    x = np.ascontiguousarray(x, float); e2 = np.ascontiguousarray(e2, float)
    out = np.empty((len(x), len(e2) - 1))
    load_quad().ora_point_cell_matrix(kq, p, q, len(x), _ptr(x), len(e2) - 1, _ptr(e2), ell, _ptr(out))
    return out


def point_point(p: int, q: int, x: np.ndarray, x2: np.ndarray, ell: float, kq: int = -1) -> np.ndarray:
    """P^{pq}[i, j] = d^p_x d^q_{x'} k(x_i, x'_j)."""
    if kq >= 0 and p + q > 2 * kq:
        raise ValueError(f"derivative order {p + q} exceeds the smoothness of Matern-{kq}+1/2")
    x = np.ascontiguousarray(x, float); x2 = np.ascontiguousarray(x2, float)
    out = np.empty((len(x), len(x2)))
    load_quad().ora_point_point_matrix(kq, p, q, len(x), _ptr(x), len(x2), _ptr(x2), ell, _ptr(out))
    return out


def _kron_all(mats: Sequence[np.ndarray]) -> np.ndarray:
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def _mode_apply(mats: Sequence[np.ndarray], v: np.ndarray, shape_in: Sequence[int]) -> np.ndarray:
    """(M_0 kron M_1 kron ...) v for a row-major tensor v of shape shape_in."""
    x = v.reshape(shape_in)
    for d, m in enumerate(mats):
        x = np.moveaxis(np.tensordot(m, x, axes=(1, d)), 0, d)
    return x.reshape(-1)


class Oracle:
    """All oracle quantities of one IBVP (``workloads.IBVP``).

    Several outputs (Sec. 3.3): the prior is k = diag(k_11, ..., k_d'd')
    (eq. multioutput-cov-def), here every k_ii the same tensor-product kernel
    times its own outputscale sigma_i^2.  A volume observation of equation e
    is sum over terms of e of c_t d^alpha_t u_out(t) integrated over the cell;
    two observations covary only through terms on the same output, so every
    Gram entry is a sum over term pairs with out(t1) = out(t2) of
    sigma_out^2 c_t1 c_t2 prod_i F^{alpha_i alpha'_i}.  Volume observations
    are ordered equation-major (all cells of equation 0 first).  A point
    observation is a sum of terms coef * w(x) * d^beta u_out(x) (one term for
    an initial or Dirichlet value, two for a radiation condition)."""

    def __init__(self, ibvp):
        self.p = ibvp
        self.d = ibvp.d
        self.ell = tuple(float(l) for l in ibvp.lengthscale)
        self.kq = tuple(kernel_q(c) for c in ibvp.kernel_codes())
        self.sfo = ibvp.output_scales()
        self.sf2 = float(self.sfo[0])
        self._cache: Dict[tuple, np.ndarray] = {}
        self.neq = ibvp.neq
        self.Nc = ibvp.n_cells
        self.N = ibvp.n_pde
        self.ncell = ibvp.ncell
        self.cc = None if ibvp.cell_coef is None else np.asarray(ibvp.cell_coef, float).ravel()

    # -- factor caches -----------------------------------------------------
    def F(self, dim: int, p: int, q: int) -> np.ndarray:
        key = ("F", dim, p, q)
        if key not in self._cache:
            e = self.p.edges[dim]
            self._cache[key] = cell_cell(p, q, e, e, self.ell[dim], self.kq[dim])
        return self._cache[key]

    def term_coef(self, term) -> np.ndarray:
        """c_alpha(V) for every cell V (Sec. 3.2; per-cell coefficients as
        in the appendix on variable bathymetry)."""
        if term.cellwise:
            return term.coef * self.cc
        return np.full(self.Nc, term.coef)

    def _rows(self, eq: int) -> slice:
        return slice(eq * self.Nc, (eq + 1) * self.Nc)

    # -- volume block (Sec. 3.2 eq. LkL, Sec. 4.1 eq. kronecker-structure) --
    def volume_gram(self) -> np.ndarray:
        """Dense L_V k L_V' (N x N), summed over every (alpha, alpha') pair
        of terms on the same output."""
        G = np.zeros((self.N, self.N))
        for t1 in self.p.terms:
            c1 = self.term_coef(t1)
            for t2 in self.p.terms:
                if t1.out != t2.out:
                    continue
                c2 = self.term_coef(t2)
                K = _kron_all([self.F(i, t1.alpha[i], t2.alpha[i]) for i in range(self.d)])
                G[self._rows(t1.eq), self._rows(t2.eq)] += self.sfo[t1.out] * (c1[:, None] * K * c2[None, :])
        return G

    def volume_diag(self) -> np.ndarray:
        diag = np.zeros(self.N)
        for t1 in self.p.terms:
            c1 = self.term_coef(t1)
            for t2 in self.p.terms:
                if t1.out != t2.out or t1.eq != t2.eq:
                    continue
                c2 = self.term_coef(t2)
                dg = [np.diag(self.F(i, t1.alpha[i], t2.alpha[i])) for i in range(self.d)]
                diag[self._rows(t1.eq)] += self.sfo[t1.out] * (c1 * c2 * _kron_all(dg))
        return diag

    def noise_pde(self) -> float:
        """PDE-observation noise variance; relative mode scales by the mean of
        the volume Gram's diagonal (reading of Sec. 2.1's Sigma)."""
        if self.p.noise_pde_relative:
            return float(self.p.noise_pde * self.volume_diag().mean())
        return float(self.p.noise_pde)

    def volume_matvec(self, v: np.ndarray) -> np.ndarray:
        """Matrix-free (L_V k L_V') v as a sum of Kronecker products."""
        y = np.zeros(self.N)
        for t1 in self.p.terms:
            c1 = self.term_coef(t1)
            for t2 in self.p.terms:
                if t1.out != t2.out:
                    continue
                c2 = self.term_coef(t2)
                mats = [self.F(i, t1.alpha[i], t2.alpha[i]) for i in range(self.d)]
                y[self._rows(t1.eq)] += self.sfo[t1.out] * (c1 * _mode_apply(mats, c2 * v[self._rows(t2.eq)],
                                                                                   self.ncell))
        return y

    # -- point observations (Sec. 2.2, IC/BC operator) -----------------------
    def point_gram(self) -> np.ndarray:
        """L_b k L_b' + Sigma_b (dense)."""
        gs = self.p.groups
        if not gs:                                   # no IC/BC observations: an empty block
            return np.zeros((0, 0))
        blocks = []
        for g1 in gs:
            row = []
            for g2 in gs:
                B = np.zeros((g1.size, g2.size))
                for c1 in g1.components():
                    for c2 in g2.components():
                        if c1.out != c2.out:
                            continue
                        mats = [point_point(c1.deriv[i], c2.deriv[i], g1.axes[i], g2.axes[i], self.ell[i], self.kq[i])
                                for i in range(self.d)]
                        w = np.outer(c1.weight_grid(g1.shape), c2.weight_grid(g2.shape))
                        B += (self.sfo[c1.out] * c1.coef * c2.coef) * (w * _kron_all(mats))
                row.append(B)
            blocks.append(row)
        G = np.block(blocks)
        G[np.diag_indices_from(G)] += np.concatenate([np.full(g.size, g.noise_var) for g in gs])
        return G

    def _group_cell_mats(self, g, beta, alpha) -> List[np.ndarray]:
        return [self.pc_cached(g, i, beta[i], alpha[i]) for i in range(self.d)]

    def pc_cached(self, g, dim, p, q):
        key = ("Q", id(g), dim, p, q)
        if key not in self._cache:
            self._cache[key] = point_cell(p, q, g.axes[dim], self.p.edges[dim], self.ell[dim], self.kq[dim])
        return self._cache[key]

    def _pairs(self, g):
        """(point term, PDE term, scale) for every pair on the same output."""
        for c in g.components():
            for t in self.p.terms:
                if t.out == c.out:
                    yield c, t, self.sfo[c.out] * c.coef

    def cross_gram(self) -> np.ndarray:
        """L_b k L_V' (n_b x N), dense."""
        rows = [np.zeros((0, self.N))]
        for g in self.p.groups:
            B = np.zeros((g.size, self.N))
            for c, t, a in self._pairs(g):
                K = _kron_all(self._group_cell_mats(g, c.deriv, t.alpha))
                B[:, self._rows(t.eq)] += a * (c.weight_grid(g.shape)[:, None] * K * self.term_coef(t)[None, :])
            rows.append(B)
        return np.vstack(rows)

    def cross_matvec(self, v: np.ndarray) -> np.ndarray:
        """(L_b k L_V') v, matrix-free per tensor-grid group."""
        out = [np.zeros(0)]
        for g in self.p.groups:
            acc = np.zeros(g.size)
            for c, t, a in self._pairs(g):
                acc += a * c.weight_grid(g.shape) * _mode_apply(self._group_cell_mats(g, c.deriv, t.alpha),
                                                                self.term_coef(t) * v[self._rows(t.eq)], self.ncell)
            out.append(acc)
        return np.concatenate(out)

    def cross_rmatvec(self, w: np.ndarray) -> np.ndarray:
        """(L_V k L_b') w = (L_b k L_V')^T w."""
        y = np.zeros(self.N)
        off = 0
        for g in self.p.groups:
            wg = w[off:off + g.size]; off += g.size
            for c, t, a in self._pairs(g):
                mats = [m.T for m in self._group_cell_mats(g, c.deriv, t.alpha)]
                y[self._rows(t.eq)] += a * self.term_coef(t) * _mode_apply(mats, c.weight_grid(g.shape) * wg, g.shape)
        return y

    def gram(self) -> np.ndarray:
        """Full IBVP Gram G = L k L' + Sigma (Sec. 2.2)."""
        Gbb = self.point_gram()
        Gbp = self.cross_gram()
        Gpp = self.volume_gram()
        Gpp[np.diag_indices_from(Gpp)] += self.noise_pde()
        return np.block([[Gbb, Gbp], [Gbp.T, Gpp]])

    # -- cross-covariances with evaluation points (Sec. 2.1 eq. Lk-def) ------
    def grid_points(self, grid: Sequence[np.ndarray]) -> np.ndarray:
        mesh = np.meshgrid(*grid, indexing="ij")
        return np.stack([m.ravel() for m in mesh], axis=1)

    def Lk_points(self, X: np.ndarray, out: int = 0) -> Tuple[np.ndarray, np.ndarray]:
        """(L_b k(x), L_V k(x)) for the value of output ``out`` at the rows x
        of X: shapes (n_b, M) and (N, M)."""
        M = X.shape[0]
        sf = self.sfo[out]
        kb = [np.zeros((0, M))]
        for g in self.p.groups:
            blk_g = np.zeros((g.size, M))
            idx = np.indices(g.shape).reshape(self.d, -1)
            for c in g.components():
                if c.out != out:
                    continue
                mats = [point_point(c.deriv[i], 0, g.axes[i], X[:, i], self.ell[i], self.kq[i]) for i in range(self.d)]
                # group tensor grid x each evaluation point: product over dims
                blk = np.ones((g.size, M))
                for i in range(self.d):
                    blk *= mats[i][idx[i], :]
                blk_g += (sf * c.coef) * (c.weight_grid(g.shape)[:, None] * blk)
            kb.append(blk_g)
        kp = np.zeros((self.N, M))
        idx = np.indices(self.ncell).reshape(self.d, -1)
        for t in self.p.terms:
            if t.out != out:
                continue
            blk = np.ones((self.Nc, M))
            for i in range(self.d):
                # L_[a,b];alpha applied to the first argument of k(., x)
                q = point_cell(0, t.alpha[i], X[:, i], self.p.edges[i], self.ell[i], self.kq[i])  # M x N_i
                blk *= q.T[idx[i], :]
            kp[self._rows(t.eq)] += sf * (self.term_coef(t)[:, None] * blk)
        return np.vstack(kb), kp


def dense_posterior(orc: Oracle, X: np.ndarray, y: Optional[np.ndarray] = None, out: int = 0):
    """Exact posterior mean/variance of output ``out`` at rows of X (Sec. 2.1
    eq. lin-cond-mean, eq. lin-cond-cov; Sec. 4 representer weights via
    Cholesky)."""
    G = orc.gram()
    y = orc.p.y_obs() if y is None else y
    cf = sla.cho_factor(G, lower=True)
    alpha = sla.cho_solve(cf, y)
    kb, kp = orc.Lk_points(X, out)
    Lk = np.vstack([kb, kp])
    mean = Lk.T @ alpha
    W = sla.solve_triangular(cf[0], Lk, lower=True)
    var = orc.sfo[out] - np.einsum("ij,ij->j", W, W)
    return mean, var, alpha


# ---------------------------------------------------------------------------
# Two-stage solve: exact IC/BC conditioning, then IterGP on the volumes
# (Sec. 4.2 Cholesky preconditioner; Sec. 4.1 IterGP)
# ---------------------------------------------------------------------------

class SchurSystem:
    """Gram of the volume observations under the IC/BC-conditioned prior:
    S = L_V k L_V' + Sigma_V - G_pb G_bb^{-1} G_bp, and its data residual."""

    def __init__(self, orc: Oracle):
        self.o = orc
        self.Gbb = orc.point_gram()
        # no IC/BC observations: nothing to condition on first, S is the volume Gram
        self.cf = sla.cho_factor(self.Gbb, lower=True) if orc.p.n_b > 0 else None
        self.sig = orc.noise_pde()
        yobs = orc.p.y_obs()
        self.yb = yobs[:orc.p.n_b]
        self.yp = yobs[orc.p.n_b:]
        self.ab0 = self.bb_solve(self.yb)                     # G_bb^{-1} y_b
        self.b = self.yp - orc.cross_rmatvec(self.ab0)        # y_p - G_pb G_bb^{-1} y_b
        self.nmv = 0

    def bb_solve(self, B: np.ndarray) -> np.ndarray:
        """G_bb^{-1} B (LAPACK Cholesky); B with n_b rows."""
        return sla.cho_solve(self.cf, B) if self.cf is not None else np.zeros(B.shape)

    def bb_lsolve(self, B: np.ndarray) -> np.ndarray:
        """L^{-1} B with G_bb = L L^T."""
        return sla.solve_triangular(self.cf[0], B, lower=True) if self.cf is not None else np.zeros(B.shape)

    def matvec(self, v: np.ndarray) -> np.ndarray:
        self.nmv += 1
        o = self.o
        w = self.bb_solve(o.cross_matvec(v))
        return o.volume_matvec(v) + self.sig * v - o.cross_rmatvec(w)

    def full_weights(self, vp: np.ndarray) -> np.ndarray:
        """Representer weights of the full system from the volume weights."""
        ab = self.bb_solve(self.yb - self.o.cross_matvec(vp))
        return np.concatenate([ab, vp])


def itergp(S, maxiter: int, tol: float = 0.0, actions: str = "cg", store: bool = True, passes: int = 1,
           init: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None):
    """IterGP (Wenger et al. 2022, as used in Sec. 4.1/4.2) on system S with
    right-hand side S.b:

        r   = b - S v          (residual of the current representer weights)
        s   = action           (CG policy: s = r; 'unit': e_i)
        z   = S s
        d   = s - C z          (C = sum_j d_j d_j^T / eta_j)
        eta = z^T d
        C  += d d^T / eta
        v  += (s^T r / eta) d

    passes = 2 repeats the projection onto the S-complement of the stored
    directions once more on d (d <- d - C S d, "full reorthogonalisation"
    done twice, Limitations section) and then takes eta = d^T S d, which equals
    z^T d in exact arithmetic.

    init = (v0, D0, eta0) continues from that state: the stored directions
    D0 (with their eta0) stay in C and the iterations add to them (maxiter
    counts the new ones).

    Returns (v, D, eta, residual norms).  Stops after maxiter iterations or
    once ||r|| <= tol ||b||."""
    b = S.b
    n = len(b)
    k0 = 0 if init is None else init[1].shape[1]
    v = np.zeros(n) if init is None else np.array(init[0], dtype=float)
    D = np.zeros((n, k0 + maxiter)) if store else None
    eta = np.zeros(k0 + maxiter)
    if k0:
        D[:, :k0] = init[1]
        eta[:k0] = init[2]
    res = []
    nb = np.linalg.norm(b)
    k = k0
    for i in range(k0, k0 + maxiter):
        r = b - S.matvec(v) if i > 0 else b.copy()
        res.append(np.linalg.norm(r))
        if tol > 0 and res[-1] <= tol * nb:
            break
        if actions == "cg":
            s = r
        elif actions == "unit":
            s = np.zeros(n); s[i] = 1.0
        else:
            raise ValueError(actions)
        z = S.matvec(s)
        d = s - D[:, :i] @ ((D[:, :i].T @ z) / eta[:i]) if i > 0 else s.copy()
        if passes == 2:
            if i > 0:
                d = d - D[:, :i] @ ((D[:, :i].T @ S.matvec(d)) / eta[:i])
            et = d @ S.matvec(d)
        else:
            et = z @ d
        if not et > 0:
            break
        D[:, i] = d
        eta[i] = et
        v = v + (s @ r) / et * d
        k = i + 1
    else:
        r = b - S.matvec(v)
        res.append(np.linalg.norm(r))
    return v, D[:, :k], eta[:k], np.array(res)


def coarse_aggregation(p, factors: Sequence[int]) -> np.ndarray:
    """The nested coarse scheme of the appendix "Multigrid preconditioners":
    coarse cell a is the union of the factors[0] x ... x factors[d-1] fine
    cells that refine it (Fig. multigrid-pyramid), so by eq.
    subdomain-partition its integral functional is the sum of theirs.
    Returns C (Nc x N, 0/1) with (C u)_a = sum of the fine values inside a,
    both flattened row-major."""
    nc = p.ncell
    f = tuple(int(x) for x in factors)
    if len(f) != p.d or any(x < 1 or n % x for x, n in zip(f, nc)):
        raise ValueError(f"coarsening factors {f} must divide the cell counts {nc}")
    cc = tuple(n // x for n, x in zip(nc, f))
    fine = np.indices(nc).reshape(p.d, -1)                 # fine multi-indices, row-major
    coarse = np.ravel_multi_index(tuple(fine[i] // f[i] for i in range(p.d)), cc)
    C = np.zeros((int(np.prod(cc)), int(np.prod(nc))))
    C[coarse, np.arange(C.shape[1])] = 1.0
    return C


def itergp_coarse(S, C: np.ndarray, maxiter: int, tol: float = 0.0, passes: int = 2):
    """Coarse-scheme warm start (appendix "Multigrid preconditioners"): first
    condition exactly on the coarse observations C y_V, then run IterGP with
    CG actions on the fine volume observations as before.

    Under the IC/BC-conditioned prior (Sec. 4.2) the coarse observations have
    the Gram C S C^T, the aggregated fine noise included.  Conditioning on
    them exactly is IterGP on S with the block of actions C^T solved by one
    Cholesky factorisation C S C^T = L L^T: the directions D0 = C^T L^{-T}
    are S-orthonormal (eta = 1) and the weights start at v0 = D0 D0^T b.
    The CG iterations then continue with D0 kept in the inverse
    approximation.  Returns (v, D, eta, residual norms of the CG phase)."""
    SC = np.stack([S.matvec(c) for c in C], axis=1)          # S C^T, N x Nc
    L = np.linalg.cholesky(C @ SC)
    D0 = sla.solve_triangular(L, C, lower=True).T            # C^T L^{-T}
    eta0 = np.ones(D0.shape[1])
    v0 = D0 @ (D0.T @ S.b)
    return itergp(S, maxiter, tol=tol, passes=passes, init=(v0, D0, eta0))


def cg_solve(S, tol: float, maxiter: int):
    """Plain conjugate gradients (Sec. 4.1) on S x = S.b."""
    b = S.b
    x = np.zeros_like(b); r = b.copy(); p = r.copy(); rr = r @ r
    nb = np.sqrt(rr)
    for it in range(maxiter):
        if np.sqrt(rr) <= tol * nb:
            return x, it
        Ap = S.matvec(p)
        a = rr / (p @ Ap)
        x += a * p; r -= a * Ap
        rr2 = r @ r
        p = r + (rr2 / rr) * p
        rr = rr2
    return x, maxiter


def schur_cross(S: "SchurSystem", X: np.ndarray, out: int = 0) -> np.ndarray:
    """Cross-covariance between the volume observations and output ``out`` at
    the points X under the IC/BC-conditioned prior (Sec. 4.2):
    K_S(X) = L_V k(X) - G_pb G_bb^{-1} L_b k(X), shape (N, M)."""
    o = S.o
    kb, kp = o.Lk_points(X, out)
    if kb.size == 0:
        return kp
    return kp - np.stack([o.cross_rmatvec(c) for c in S.bb_solve(kb).T], axis=1)


def itergp_targeted(S, vp: np.ndarray, D: np.ndarray, eta: np.ndarray, KS: np.ndarray, betas: np.ndarray,
                    passes: int = 2):
    """Targeted uncertainty reduction (appendix "Targeted uncertainty
    reduction"): IterGP continued from (vp, D, eta), where iteration i takes as
    its action the residual of the right-hand side b_i = KS @ betas[i] with
    respect to the current inverse approximation C = D diag(1/eta) D^T,

        s = b_i - S C b_i,

    and otherwise the IterGP step of ``itergp`` (projection against the stored
    directions, once or twice; eta; representer weights updated with the data
    residual).  The weights betas (one row per iteration, e.g. Dirichlet draws)
    are inputs.  Returns (v, D, eta, norms of the action residuals)."""
    v = vp.copy()
    Ds = [D[:, j] for j in range(D.shape[1])]
    es = list(eta)
    res = []
    for beta in betas:
        bt = KS @ beta
        Dm = np.stack(Ds, axis=1) if Ds else np.zeros((len(v), 0))
        e = np.asarray(es)
        s = bt - S.matvec(Dm @ ((Dm.T @ bt) / e)) if Ds else bt.copy()
        res.append(np.linalg.norm(s))
        z = S.matvec(s)
        d = s - Dm @ ((Dm.T @ z) / e) if Ds else s.copy()
        if passes == 2:
            if Ds:
                d = d - Dm @ ((Dm.T @ S.matvec(d)) / e)
            et = d @ S.matvec(d)
        else:
            et = z @ d
        if not et > 0:
            break
        r = S.b - S.matvec(v)
        v = v + (d @ r) / et * d
        Ds.append(d)
        es.append(et)
    return v, np.stack(Ds, axis=1), np.asarray(es), np.asarray(res)


def two_stage_posterior(S: SchurSystem, vp: np.ndarray, X: np.ndarray,
                        D: Optional[np.ndarray] = None, eta: Optional[np.ndarray] = None, out: int = 0):
    """Posterior mean, and (if D, eta given) IterGP combined variance, of
    output ``out`` at the rows of X from volume weights vp (Sec. 4.2; Wenger
    et al. 2022 combined covariance k - k_x^T C k_x under the IC/BC-conditioned
    prior)."""
    o = S.o
    kb, kp = o.Lk_points(X, out)
    alpha = S.full_weights(vp)
    mean = kb.T @ alpha[:o.p.n_b] + kp.T @ alpha[o.p.n_b:]
    if D is None:
        return mean, None
    Wb = S.bb_lsolve(kb)
    var_b = o.sfo[out] - np.einsum("ij,ij->j", Wb, Wb)
    # cross-covariance of the conditioned prior between volumes and x
    w = kp - np.stack([o.cross_rmatvec(c) for c in S.bb_solve(kb).T], axis=1)
    proj = D.T @ w                                   # k x M
    var = var_b - np.einsum("ij,ij->j", proj, proj / eta[:, None])
    return mean, var
