"""The allocation-free volume-Gram matvec (gpfvm_volume_matvec_noalloc, for
callers that cannot allocate device memory) against the allocating entry point
gpfvm_volume_matvec, through the C-ABI: the same plan and kernels, so the same
bits; two calls in a row on one GPU, the second with a smaller input; sizes
beyond the static scratch refused on the host."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_05020_amd as G
    G.lib()
    return G


def _both(G, p, nrhs, seed):
    rng = np.random.default_rng(seed)
    x = torch.as_tensor(rng.standard_normal(nrhs * p.n_pde), device="cuda:0")
    y_ref = torch.empty_like(x)
    y_na = torch.full_like(x, np.nan)
    h = G.assemble(p, max_iter=4)
    try:
        G.volume_matvec(h, x, y_ref, nrhs=nrhs)
        G.volume_matvec_noalloc(h, x, y_na, nrhs=nrhs)
        torch.cuda.synchronize()
        return y_ref.cpu().numpy(), y_na.cpu().numpy()
    finally:
        G.destroy(h)


def test_noalloc_equals_allocating_matvec_twice(G):
    # first a larger call (3-D, per-cell coefficients, 8 rhs), then a smaller one (2-D, 1 rhs)
    for p, nrhs, seed in [(W.wave2d_c4(nt=8, nx=40, ny=33, n_ic=10, n_bt=4, n_bs=6), 8, 1),
                          (W.advdiff_c2(nt=37, nx=45, n_ic=50), 1, 2)]:
        ref, got = _both(G, p, nrhs, seed)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref), (p.name, nrhs, float(np.max(np.abs(got - ref))))


def test_noalloc_refuses_sizes_beyond_the_scratch(G):
    p = W.wave2d_c4()                       # 1 048 576 volumes: the plan needs far more than the scratch
    h = G.assemble(p, max_iter=1)
    try:
        x = torch.zeros(p.n_pde, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        with pytest.raises(G.GpfvmError) as e:
            G.volume_matvec_noalloc(h, x, y)
        assert e.value.code == G.E_INVALID and "scratch" in str(e.value)
        # the handle still works afterwards, through the allocation-free path too
        q = W.advdiff_c2(nt=12, nx=10, n_ic=20)
        ref, got = _both(G, q, 2, 3)
        assert np.array_equal(got, ref)
    finally:
        G.destroy(h)
