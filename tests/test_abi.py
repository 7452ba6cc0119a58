"""CPU tests of the C-ABI boundary: the library loads, exports every entry
point that include/gpfvm.h declares, and rejects malformed IBVPs before any
HIP call (argument validation runs on the host)."""
import dataclasses
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "gpfvm.h")).read()
    return sorted(set(re.findall(r"\b(gpfvm_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def G():
    import paper_2406_05020_amd as G
    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libgpfvm.so not built")
    return G


def test_every_declared_symbol_is_exported(G):
    L = G.lib()
    names = _declared()
    assert "gpfvm_assemble" in names and "gpfvm_posterior" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(G.SYMBOLS), set(names) ^ set(G.SYMBOLS)


def test_valid_workloads_pass_validation(G):
    for p in (W.heat1d_c1(), W.advdiff_c2(nt=8, nx=8), W.heat2d_c3(nt=4, nx=4, ny=4),
              W.wave2d_c4(nt=4, nx=4, ny=4)):
        G.validate(p)


@pytest.mark.parametrize("mutate, msg", [
    (lambda p: setattr(p, "d", 4), "dim"),
    (lambda p: p.edges.__setitem__(1, np.array([0.0, 0.5, 0.4, 1.0])), "increasing"),
    (lambda p: setattr(p, "lengthscale", (0.2, -0.1)), "lengthscale"),
    (lambda p: setattr(p, "outputscale", 0.0), "outputscale"),
    (lambda p: setattr(p, "noise_pde", 0.0), "noise_pde"),
    (lambda p: p.terms.append(W.PDETerm((5, 0), 1.0)), "derivative order"),
    (lambda p: p.terms.append(W.PDETerm((0, 1), 1.0, True)), "cell_coef"),
    (lambda p: setattr(p.groups[0], "noise_var", -1.0), "noise_var"),
    (lambda p: p.groups[0].y.__setitem__(0, np.nan), "not finite"),
    (lambda p: p.edges.__setitem__(0, np.array([0.0, np.inf])), "not finite"),
])
def test_invalid_ibvp_rejected_on_host(G, mutate, msg):
    p = W.heat1d_c1(nt=4, nx=4, n_ic=4)
    mutate(p)
    with pytest.raises(G.GpfvmError) as e:
        G.validate(p)
    assert e.value.code == G.E_INVALID
    assert msg in str(e.value)
    # assemble validates before touching the GPU, so the same error comes back
    with pytest.raises(G.GpfvmError) as e2:
        G.assemble(p, stream=0)
    assert e2.value.code == G.E_INVALID


def test_factor_argument_checks(G):
    import ctypes as C
    L = G.lib()
    a = np.array([0.0, 0.5, 1.0])
    p = a.ctypes.data_as(C.POINTER(C.c_double))
    assert L.gpfvm_factor(3, 0, 0, 0, 2, p, 2, p, 0.1, None, None) == G.E_INVALID
    assert L.gpfvm_factor(0, 0, 5, 5, 2, p, 2, p, 0.1, None, None) == G.E_INVALID
    assert L.gpfvm_factor(0, 0, 0, 0, 2, p, 2, p, -0.1, C.c_void_p(8), None) == G.E_INVALID
    assert "lengthscale" in G.last_error()
    assert L.gpfvm_factor(0, 7, 0, 0, 2, p, 2, p, 0.1, C.c_void_p(8), None) == G.E_INVALID
    assert "kernel" in G.last_error()
    # Matern-3/2 (q = 1) admits orders up to 1
    assert L.gpfvm_factor(0, G.KERNEL_MATERN32, 2, 0, 2, p, 2, p, 0.1, C.c_void_p(8), None) == G.E_INVALID
    assert "Matern" in G.last_error()


def test_null_handle_calls_are_rejected(G):
    import ctypes as C
    L = G.lib()
    assert L.gpfvm_matvec(None, 1, None, None, 0, 0, None) == G.E_INVALID
    assert L.gpfvm_solve(None, None, None, None) == G.E_INVALID
    assert L.gpfvm_posterior(None, 2, None, None, None, None, None) == G.E_INVALID
    L.gpfvm_destroy(None)   # accepted
    assert isinstance(G.last_error(None), str)


def test_assemble_option_checks_happen_on_the_host(G):
    """Only the float32 tile format exists; max_iter is bounded.  Both are
    rejected before any device call."""
    p = W.heat1d_c1()
    with pytest.raises(G.GpfvmError) as e:
        G.assemble(p, tile=3, stream=0)
    assert e.value.code == G.E_INVALID and "tile" in str(e.value)
    with pytest.raises(G.GpfvmError) as e:
        G.assemble(p, max_iter=0, stream=0)
    assert e.value.code == G.E_INVALID and "max_iter" in str(e.value)


def test_matern_orders_are_validated_on_the_host(G):
    """A Matern-(q+1/2) dimension admits PDE and point derivative orders up to q."""
    import dataclasses
    p = W.heat1d_c1()                                  # u_t - 0.1 u_xx: orders (1, 0) and (0, 2)
    ok = dataclasses.replace(p, kernel=(G.KERNEL_MATERN32, G.KERNEL_MATERN52))
    G.validate(ok)
    for bad in [(G.KERNEL_MATERN32, G.KERNEL_MATERN32), (G.KERNEL_MATERN12, G.KERNEL_MATERN52), (9, 0)]:
        with pytest.raises(G.GpfvmError) as e:
            G.validate(dataclasses.replace(p, kernel=bad))
        assert e.value.code == G.E_INVALID


def _small_system():
    return W.shallow_water(nt=2, nx=3, ny=4, n_icx=2, n_icy=3, n_bt=2, n_bx=2, n_by=2, grid_t=2)


def test_systems_pass_validation(G):
    G.validate(_small_system())
    G.validate(W.shallow_water())


def _set_term(p, k, **kw):
    p.terms[k] = dataclasses.replace(p.terms[k], **kw)


@pytest.mark.parametrize("mutate, msg", [
    (lambda p: _set_term(p, 0, out=3), "term_out"),
    (lambda p: _set_term(p, 0, eq=5), "term_eq"),
    (lambda p: setattr(p, "out_scale", (1.0, -2.0, 2.0)), "out_scale"),
    (lambda p: setattr(p, "terms", [t for t in p.terms if t.eq != 2]), "equation 2 has no term"),
    (lambda p: setattr(p.groups[0], "out", 3), "output out of range"),
    (lambda p: setattr(p, "terms", [t for t in p.terms if t.out != 2] + [W.PDETerm((1, 0, 0), 1.0, False, 0, 2)]),
     "appears in no equation"),
    (lambda p: p.groups[3].terms.append(W.PointTerm((0, 0, 0), 1.0, 0)), "nterm out of range"),
    (lambda p: setattr(p.groups[3].terms[1], "weights", [None, None, np.array([np.nan, 1.0])]), "weight not finite"),
    (lambda p: setattr(p.groups[3].terms[1], "deriv", (0, 3, 0)), "derivative order"),
])
def test_invalid_systems_rejected_on_host(G, mutate, msg):
    p = _small_system()
    mutate(p)
    with pytest.raises(G.GpfvmError) as e:
        G.validate(p)
    assert e.value.code == G.E_INVALID
    assert msg in str(e.value), str(e.value)


def test_binding_checks_array_lengths(G):
    """The library reads neq x cells values of f_int and one value per cell of
    cell_coef through plain pointers; the binding refuses arrays of another length."""
    p = _small_system()
    p.f_int = np.zeros(p.n_cells)               # one equation's worth for three equations
    with pytest.raises(ValueError):
        G.validate(p)
    p = _small_system()
    p.cell_coef = np.ones(p.n_cells + 1)
    with pytest.raises(ValueError):
        G.validate(p)
