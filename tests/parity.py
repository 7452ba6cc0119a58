"""Comparison helpers shared by the GPU parity tests.

A posterior quantity (mean or variance on a grid) passes when both the
L2-relative error over the points and the largest absolute error, normalised
by the prior variance sf2 or by the quantity's own largest magnitude if that
is larger, are within the tolerance: the norm alone would let one entry among
tens of thousands be off by far more than the bound.  (An early-terminated
IterGP mean can exceed the data by an order of magnitude; its pointwise
error is then measured against that scale.)

Comparisons of the same recurrences (a fixed number of IterGP iterations on
both sides) hold the largest error to the L2 bound.  Comparisons of two
solves that each stopped at a residual tolerance (against a Cholesky
posterior, or two different iterative paths) differ by the unresolved part of
the solution, which the residual bounds only in norm; those pass
CONVERGED_MAXABS = 10 x the L2 bound pointwise.
"""

CONVERGED_MAXABS = 10.0
import numpy as np


def relerr(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def maxabs(a, b, sf2=1.0):
    """max |a - b| / max(sf2, max |b|)"""
    a, b = np.ravel(a), np.ravel(b)
    if not a.size:
        return 0.0
    return float(np.max(np.abs(a - b))) / max(sf2, float(np.max(np.abs(b))))


def assert_close(got, ref, tol, sf2=1.0, what="", converged=False):
    """Element-wise and L2 agreement of a posterior mean or variance
    (converged=True: two solves stopped at a residual tolerance)."""
    got, ref = np.ravel(got), np.ravel(ref)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), (what, "non-finite values")
    e2, ea = relerr(got, ref), maxabs(got, ref, sf2)
    ta = tol * (CONVERGED_MAXABS if converged else 1.0)
    assert e2 <= tol and ea <= ta, (what, "L2-relative", e2, "max-abs/sf2", ea, "tols", tol, ta)
