"""Pins of the oracle's half-integer Matern factors (Sec. 3.1: nu = q + 1/2,
k(r) = exp(-c|r|/l) p_q(c|r|/l), c = sqrt(2q + 1)), independent of the
oracle's own derivative code: textbook closed forms differentiated by sympy,
mpmath quadrature split at the kinks, and identities of the cell integrals."""
import mpmath as mp
import numpy as np
import pytest
import sympy as sp

from oracle import gpfvm_oracle as O

R = sp.symbols("r", positive=True)
L = sp.symbols("l", positive=True)
# Rasmussen & Williams eq. 4.17 (nu = 3/2, 5/2) and the nu = 7/2 member, written out
TEXTBOOK = {
    1: (1 + sp.sqrt(3) * R / L) * sp.exp(-sp.sqrt(3) * R / L),
    2: (1 + sp.sqrt(5) * R / L + sp.Rational(5, 3) * R**2 / L**2) * sp.exp(-sp.sqrt(5) * R / L),
    3: (1 + sp.sqrt(7) * R / L + sp.Rational(14, 5) * R**2 / L**2 + sp.Rational(7, 15) * sp.sqrt(7) * R**3 / L**3)
    * sp.exp(-sp.sqrt(7) * R / L),
}


def kder_ref(q, m, r, l):
    """m-th derivative of the textbook Matern kernel at r != 0 (even in r)."""
    f = sp.diff(TEXTBOOK[q], R, m).subs({L: l})
    v = float(f.subs(R, abs(r)))
    return -v if (m % 2 and r < 0) else v


@pytest.mark.parametrize("q", [1, 2, 3])
def test_matern_derivatives_match_sympy(q):
    lib = O.load_quad()
    for m in range(0, 2 * q + 1):
        for r in (-0.37, -0.05, 0.012, 0.2, 0.9):
            ref = kder_ref(q, m, r, 0.3)
            got = lib.ora_kder_k(q, m, r, 0.3)
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (q, m, r, got, ref)


def _mp_kder(q, m, l):
    f = sp.lambdify(R, sp.diff(TEXTBOOK[q], R, m).subs({L: l}), "mpmath")
    return lambda r: f(abs(r)) * (-1 if (m % 2 and r < 0) else 1)


@pytest.mark.parametrize("q,p,qq", [(1, 0, 0), (1, 1, 1), (2, 0, 2), (2, 2, 1), (3, 1, 2)])
def test_matern_point_cell_matches_mpmath(q, p, qq):
    mp.mp.dps = 25
    l, x, a, b = 0.25, 0.31, 0.1, 0.45          # x inside the cell: kink at s' = x
    g = _mp_kder(q, p + qq, l)
    ref = float((-1) ** qq * (mp.quad(lambda s2: g(x - s2), [a, x]) + mp.quad(lambda s2: g(x - s2), [x, b])))
    got = O.point_cell(p, qq, np.array([x]), np.array([a, b]), l, kq=q)[0, 0]
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (got, ref)


@pytest.mark.parametrize("q,p,qq,I,J", [(1, 0, 0, (0.0, 0.2), (0.1, 0.35)),
                                         (2, 1, 1, (0.0, 0.2), (0.1, 0.35)),
                                         (2, 2, 0, (0.0, 0.15), (0.3, 0.5)),
                                         (2, 2, 2, (0.0, 0.2), (0.05, 0.3))])
def test_matern_cell_cell_matches_mpmath(q, p, qq, I, J):
    mp.mp.dps = 20
    l = 0.3
    g = _mp_kder(q, p + qq, l)

    def inner(s):
        pts = sorted({J[0], J[1], min(max(s, J[0]), J[1])})
        return mp.quad(lambda s2: g(s - s2), pts)

    cuts = sorted({I[0], I[1]} | {c for c in J if I[0] < c < I[1]})
    ref = float((-1) ** qq * mp.quad(inner, cuts))
    got = O.cell_cell(p, qq, np.array(I), np.array(J), l, kq=q)[0, 0]
    assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref)), (got, ref)


@pytest.mark.parametrize("q", [1, 2, 3])
def test_matern_cell_identities(q):
    l, h = 0.2, 0.07
    kh = float(TEXTBOOK[q].subs({L: l, R: h}))
    # F^{11}(I, I) = 2 (k(0) - k(h)) for any stationary kernel with k(0) = 1
    f11 = O.cell_cell(1, 1, np.array([0.0, h]), np.array([0.0, h]), l, kq=q)[0, 0]
    assert abs(f11 - 2.0 * (1.0 - kh)) <= 1e-12
    # l -> infinity: k -> 1, F^{00} -> |I| |J|
    f00 = O.cell_cell(0, 0, np.array([0.0, 0.3]), np.array([0.5, 0.6]), 1e6, kq=q)[0, 0]
    assert abs(f00 - 0.03) <= 1e-6
    # Gram symmetry: F^{pq}(I, J) = F^{qp}(J, I)
    e = np.array([0.0, 0.1, 0.25, 0.3])
    for p, qq in [(1, 0), (q, 1), (0, q)]:
        A = O.cell_cell(p, qq, e, e, l, kq=q)
        B = O.cell_cell(qq, p, e, e, l, kq=q)
        assert np.abs(A - B.T).max() <= 1e-12 * np.abs(A).max()


def test_matern_order_beyond_smoothness_is_refused():
    with pytest.raises(ValueError):
        O.cell_cell(2, 2, np.array([0.0, 0.1]), np.array([0.0, 0.1]), 0.2, kq=1)
    with pytest.raises(ValueError):
        O.point_point(2, 1, np.array([0.0]), np.array([0.1]), 0.2, kq=1)
