"""Pins of the oracle's 1-D quadrature factors against things other than itself:
the Gauss-Kronrod rule's polynomial exactness, symbolic derivatives (sympy),
high-precision quadrature (mpmath), the closed-form antiderivative reduction
of Sec. 3.1 eq. linop-simplified written out independently here, and special
cases with textbook values."""
import math

import mpmath
import numpy as np
import pytest
import sympy as sp

from oracle import gpfvm_oracle as O


def test_qk15_polynomial_exactness():
    lib = O.load_quad()
    import ctypes
    k_, g_ = ctypes.c_double(), ctypes.c_double()
    a, b = -0.3, 1.7
    for k in range(0, 23):
        lib.ora_qk15_monomial(k, a, b, ctypes.byref(k_), ctypes.byref(g_))
        exact = (b ** (k + 1) - a ** (k + 1)) / (k + 1)
        assert abs(k_.value - exact) <= 1e-13 * max(1.0, abs(exact)), k
        if k <= 13:   # 7-point Gauss is exact through degree 13
            assert abs(g_.value - exact) <= 1e-13 * max(1.0, abs(exact)), k
    # and Gauss-7 is *not* exact at degree 14 (catches a swapped weight table)
    lib.ora_qk15_monomial(14, a, b, ctypes.byref(k_), ctypes.byref(g_))
    assert abs(g_.value - (b ** 15 - a ** 15) / 15) > 1e-10


@pytest.mark.parametrize("m", range(0, 7))
def test_kernel_derivative_matches_sympy(m):
    r, l = sp.symbols("r l", real=True)
    f = sp.lambdify((r, l), sp.diff(sp.exp(-r ** 2 / (2 * l ** 2)), r, m), "math")
    lib = O.load_quad()
    for rv in (-0.7, -0.13, 0.0, 0.05, 0.41):
        for lv in (0.1, 0.3):
            ref = f(rv, lv)
            got = lib.ora_kder(m, rv, lv)
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)) * (1 / lv) ** m


def _closed_form_cell_cell(p, q, a, b, a2, b2, l):
    """Independent closed form: by the fundamental theorem of calculus on both
    sides, F^{pq} = (-1)^q [g(b-a2) - g(a-a2) - g(b-b2) + g(a-b2)] with g the
    (p+q-2)-th derivative (antiderivative for negative orders) of
    exp(-r^2/(2 l^2)); antiderivatives written with erf."""
    m = p + q - 2

    def g(r):
        z = r / (math.sqrt(2) * l)
        if m == -2:
            return l * math.sqrt(math.pi / 2) * r * math.erf(z) + l * l * math.exp(-z * z)
        if m == -1:
            return l * math.sqrt(math.pi / 2) * math.erf(z)
        rr = sp.symbols("rr")
        return float(sp.diff(sp.exp(-rr ** 2 / (2 * l ** 2)), rr, m).subs(rr, r))

    val = g(b - a2) - g(a - a2) - g(b - b2) + g(a - b2)
    return -val if q % 2 else val


PAIRS = [(0, 0), (1, 0), (0, 1), (1, 1), (2, 0), (0, 2), (2, 1), (1, 2), (2, 2), (4, 0), (0, 4), (3, 1)]
INTERVALS = [
    ((0.0, 0.0625), (0.0, 0.0625)),        # identical
    ((0.0, 0.0625), (0.0625, 0.125)),      # adjacent
    ((0.1, 0.2), (0.55, 0.7)),             # distant, unequal widths
    ((0.3, 0.5), (0.35, 0.45)),            # nested
]


@pytest.mark.parametrize("pq", PAIRS)
def test_cell_cell_vs_closed_form(pq):
    p, q = pq
    for (I, J) in INTERVALS:
        for l in (0.1, 0.2, 0.3):
            got = O.cell_cell(p, q, np.array(I), np.array(J), l)[0, 0]
            ref = _closed_form_cell_cell(p, q, I[0], I[1], J[0], J[1], l)
            scale = (I[1] - I[0]) * (J[1] - J[0]) * l ** (-(p + q))
            assert abs(got - ref) <= 1e-11 * scale, (I, J, l, got, ref)


def test_cell_cell_vs_mpmath():
    mpmath.mp.dps = 30
    r, l = sp.symbols("r l")
    for (p, q) in [(0, 0), (1, 1), (2, 2), (0, 3)]:
        expr = sp.diff(sp.exp(-r ** 2 / (2 * l ** 2)), r, p + q) * (-1) ** q
        f = sp.lambdify((r, l), expr, "mpmath")
        for (I, J) in INTERVALS[1:3]:
            lv = mpmath.mpf("0.2")
            ref = mpmath.quad(lambda s, s2: f(s - s2, lv), [I[0], I[1]], [J[0], J[1]])
            got = O.cell_cell(p, q, np.array(I), np.array(J), 0.2)[0, 0]
            assert abs(got - float(ref)) <= 1e-12 * max(1.0, abs(float(ref))) * 0.2 ** (-(p + q)), (p, q)


def test_point_cell_ftc_and_special_cases():
    # FTC (Sec. 3.1 eq. linop-simplified): int_a^b d/ds' k(x, s') ds' = k(x,b) - k(x,a)
    x, a, b, l = 0.37, 0.1, 0.3, 0.15
    k = lambda u, v: math.exp(-(u - v) ** 2 / (2 * l * l))
    got = O.point_cell(0, 1, np.array([x]), np.array([a, b]), l)[0, 0]
    assert abs(got - (k(x, b) - k(x, a))) < 1e-14
    # second derivative in s' integrates to the difference of first derivatives
    dk = lambda u, v: (u - v) / l ** 2 * k(u, v)      # d/dv k(u, v)
    got2 = O.point_cell(0, 2, np.array([x]), np.array([a, b]), l)[0, 0]
    assert abs(got2 - (dk(x, b) - dk(x, a))) < 1e-12
    # identical cells: F^{11}(I,I) = 2 (1 - k(h))
    h = 0.0625
    f11 = O.cell_cell(1, 1, np.array([0.0, h]), np.array([0.0, h]), l)[0, 0]
    assert abs(f11 - 2 * (1 - math.exp(-h * h / (2 * l * l)))) < 1e-14
    # very long lengthscale: F^{00} -> |I| |I'|
    f00 = O.cell_cell(0, 0, np.array([0.0, 0.3]), np.array([0.5, 0.6]), 1e4)[0, 0]
    assert abs(f00 - 0.3 * 0.1) < 1e-9
    # odd total order is antisymmetric under swapping the cells
    A = O.cell_cell(1, 0, np.array([0.0, 0.1, 0.25]), np.array([0.0, 0.1, 0.25]), 0.2)
    assert np.allclose(A, -A.T, atol=1e-15)


def test_point_point_sign_rule():
    l = 0.25
    x, x2 = 0.3, 0.1
    # d/dx' k(x, x') = (x - x')/l^2 k
    kv = math.exp(-(x - x2) ** 2 / (2 * l * l))
    got = O.point_point(0, 1, np.array([x]), np.array([x2]), l)[0, 0]
    assert abs(got - (x - x2) / l ** 2 * kv) < 1e-13
    got = O.point_point(1, 0, np.array([x]), np.array([x2]), l)[0, 0]
    assert abs(got + (x - x2) / l ** 2 * kv) < 1e-13
