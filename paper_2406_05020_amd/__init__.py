"""Python binding of the gpfvm C-ABI (libgpfvm.so): argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory and
streams.  The names follow the C entry points declared in include/gpfvm.h
(gpfvm_assemble -> assemble, ...).  Importing this module does not touch the
GPU; loading the library fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# GPFVM_LIB names another build of the same library (the host-AddressSanitizer build of asan_check.py)
LIB_PATH = os.environ.get("GPFVM_LIB") or os.path.join(HERE, "libgpfvm.so")

OK, E_INVALID, E_NOMEM, E_HIP, E_NOTPD, E_NOCONV, E_STATE = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_MIXED = 0, 1
TILE_FP32, TILE_BF16X3 = 0, 1      # low-precision volume-Gram tile formats
METHOD_ITERGP, METHOD_CG = 0, 1
DTYPE_F64, DTYPE_F32 = 0, 1
MAX_DIM, MAX_TERMS, MAX_GROUPS, MAX_OUTPUTS, MAX_PTERMS = 3, 16, 16, 8, 2
ERR_NAMES = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "HIP", -4: "NOTPD", -5: "NOCONV", -6: "STATE"}

_dp = C.POINTER(C.c_double)


class PointTerm(C.Structure):
    _fields_ = [("deriv", C.c_int * MAX_DIM), ("coef", C.c_double), ("output", C.c_int), ("weight", _dp * MAX_DIM)]


class PointGroup(C.Structure):
    _fields_ = [("n", C.c_int * MAX_DIM), ("axis", _dp * MAX_DIM), ("deriv", C.c_int * MAX_DIM),
                ("y", _dp), ("noise_var", C.c_double), ("output", C.c_int), ("nterm", C.c_int),
                ("terms", C.POINTER(PointTerm))]


class IBVPStruct(C.Structure):
    _fields_ = [("dim", C.c_int), ("ncell", C.c_int * MAX_DIM), ("edges", _dp * MAX_DIM),
                ("lengthscale", C.c_double * MAX_DIM), ("kernel", C.c_int * MAX_DIM), ("outputscale", C.c_double),
                ("nterm", C.c_int),
                ("alpha", C.POINTER(C.c_int)), ("coef", _dp), ("cellwise", C.POINTER(C.c_int)),
                ("cell_coef", _dp), ("f_int", _dp), ("noise_pde", C.c_double), ("noise_pde_relative", C.c_int),
                ("ngroup", C.c_int), ("groups", C.POINTER(PointGroup)),
                ("nout", C.c_int), ("neq", C.c_int), ("term_out", C.POINTER(C.c_int)),
                ("term_eq", C.POINTER(C.c_int)), ("out_scale", _dp)]


class AssembleOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("tile", C.c_int), ("reuse_memory", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("prec", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int), ("resume", C.c_int),
                ("tile", C.c_int), ("block", C.c_int), ("max_outer", C.c_int), ("check_every", C.c_int),
                ("reorth_passes", C.c_int), ("replace_every", C.c_int), ("coarsen", C.c_int * 3),
                ("method", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer", C.c_int), ("rel_res", C.c_double), ("rel_res_full", C.c_double),
                ("status", C.c_int), ("coarse", C.c_int)]


class HandleInfo(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_pde", C.c_longlong), ("n_b", C.c_int), ("n", C.c_longlong),
                ("noise_pde_var", C.c_double), ("device_bytes", C.c_longlong), ("volume_launches", C.c_int),
                ("volume_flops", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("workers", C.c_int), ("hbm_budget", C.c_longlong), ("prec", C.c_int), ("tol", C.c_double),
                ("max_iter", C.c_int), ("check_every", C.c_int), ("coarse_cells", C.c_int), ("max_batch", C.c_int)]


class RequestResult(C.Structure):
    _fields_ = [("rc", C.c_int), ("info", SolveInfo), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double), ("est_bytes", C.c_longlong), ("n_grid", C.c_longlong), ("batch", C.c_int)]


class ServerInfo(C.Structure):
    _fields_ = [("queued", C.c_longlong), ("completed", C.c_longlong), ("in_flight", C.c_int),
                ("peak_in_flight", C.c_int), ("reserved_bytes", C.c_longlong), ("peak_reserved_bytes", C.c_longlong),
                ("cached_bytes", C.c_longlong), ("device_bytes", C.c_longlong)]


_lib = None

SYMBOLS = {
    "gpfvm_default_assemble_opts": ([C.POINTER(AssembleOpts)], None),
    "gpfvm_default_solve_opts": ([C.POINTER(SolveOpts)], None),
    "gpfvm_validate": ([C.POINTER(IBVPStruct)], C.c_int),
    "gpfvm_assemble": ([C.POINTER(IBVPStruct), C.POINTER(AssembleOpts), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "gpfvm_matvec": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p], C.c_int),
    "gpfvm_volume_matvec": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "gpfvm_volume_matvec_noalloc": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "gpfvm_schur_matvec": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "gpfvm_solve": ([C.c_void_p, C.POINTER(SolveOpts), C.POINTER(SolveInfo), C.c_void_p], C.c_int),
    "gpfvm_posterior": ([C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(_dp), C.c_void_p, C.c_void_p,
                         C.c_void_p], C.c_int),
    "gpfvm_weights": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "gpfvm_refine_variance": ([C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(_dp), C.c_int, _dp,
                               C.POINTER(SolveInfo), C.c_void_p], C.c_int),
    "gpfvm_gram_block": ([C.c_void_p, C.c_longlong, C.c_longlong, C.c_longlong, C.c_longlong, C.c_void_p,
                          C.c_longlong, C.c_void_p], C.c_int),
    "gpfvm_factor": ([C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _dp, C.c_int, _dp, C.c_double, C.c_void_p,
                      C.c_void_p],
                     C.c_int),
    "gpfvm_get_info": ([C.c_void_p, C.POINTER(HandleInfo)], C.c_int),
    "gpfvm_default_server_opts": ([C.POINTER(ServerOpts)], None),
    "gpfvm_server_create": ([C.POINTER(ServerOpts), C.POINTER(C.c_void_p)], C.c_int),
    "gpfvm_server_submit": ([C.c_void_p, C.POINTER(IBVPStruct), C.c_int, C.POINTER(C.c_int), C.POINTER(_dp),
                             C.POINTER(C.c_longlong)], C.c_int),
    "gpfvm_server_poll": ([C.c_void_p, C.c_longlong, C.c_int, C.POINTER(C.c_int), C.POINTER(RequestResult), _dp, _dp],
                          C.c_int),
    "gpfvm_server_stats": ([C.c_void_p, C.POINTER(ServerInfo)], C.c_int),
    "gpfvm_server_destroy": ([C.c_void_p], None),
    "gpfvm_destroy": ([C.c_void_p], None),
    "gpfvm_last_error": ([C.c_void_p], C.c_char_p),
    "gpfvm_release_cached_memory": ([], C.c_longlong),
}


class GpfvmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gpfvm error {ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    """The loaded HIP library; raises if it was not built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"gpfvm HIP library not built: {LIB_PATH} is missing "
                               "(build it with: python paper_2406_05020_amd/build.py)")
        # PyTorch-ROCm ships its own HIP runtime and rocBLAS under the system libraries'
        # sonames; loaded after this library they would come in as second copies (two HIP
        # runtimes in one process).  Loading torch first makes the library bind to its copies.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SYMBOLS.items():
            f = getattr(L, name)
            f.argtypes, f.restype = args, res
        _lib = L
    return _lib


def release_cached_memory() -> int:
    """Return the unused blocks of the per-device caches to the runtime (bytes freed)."""
    return int(lib().gpfvm_release_cached_memory())


def last_error(h=None) -> str:
    return lib().gpfvm_last_error(h).decode()


def _check(rc: int, h=None):
    if rc != OK:
        raise GpfvmError(rc, last_error(h))


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


def _arr(a, dtype=np.float64):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class _Marshal:
    """Keeps the numpy buffers referenced by an IBVPStruct alive."""

    def __init__(self, p):
        self.keep = []
        s = IBVPStruct()
        s.dim = int(p.d)
        d = min(int(p.d), MAX_DIM, len(p.edges))     # the library validates dim itself
        for i in range(d):
            e = self._keep(_arr(p.edges[i]))
            s.ncell[i] = len(e) - 1
            s.edges[i] = e.ctypes.data_as(_dp)
            s.lengthscale[i] = float(p.lengthscale[i])
            s.kernel[i] = int(p.kernel_codes()[i]) if i < p.d else 0
        s.outputscale = float(p.outputscale)
        terms = list(p.terms)
        s.nterm = len(terms)
        al = self._keep(np.array([t.alpha for t in terms], dtype=np.int32).reshape(-1))
        cf = self._keep(_arr([t.coef for t in terms]))
        cw = self._keep(np.array([1 if t.cellwise else 0 for t in terms], dtype=np.int32))
        s.alpha = al.ctypes.data_as(C.POINTER(C.c_int))
        s.coef = cf.ctypes.data_as(_dp)
        s.cellwise = cw.ctypes.data_as(C.POINTER(C.c_int))
        # the library reads cells values of cell_coef and neq x cells of f_int: check the lengths here
        cells = int(np.prod([s.ncell[i] for i in range(d)]))
        neq_ = max(1, int(getattr(p, "neq", 1)))
        if getattr(p, "cell_coef", None) is not None:
            cc = self._keep(_arr(p.cell_coef).ravel())
            if cc.size != cells:
                raise ValueError(f"cell_coef holds {cc.size} values, the cells are {cells}")
            s.cell_coef = cc.ctypes.data_as(_dp)
        if getattr(p, "f_int", None) is not None:
            fi = self._keep(_arr(p.f_int).ravel())
            if fi.size != neq_ * cells:
                raise ValueError(f"f_int holds {fi.size} values, the volume observations are {neq_ * cells}")
            s.f_int = fi.ctypes.data_as(_dp)
        s.noise_pde = float(p.noise_pde)
        s.noise_pde_relative = 1 if p.noise_pde_relative else 0
        nout, neq = int(getattr(p, "nout", 1)), int(getattr(p, "neq", 1))
        s.nout, s.neq = nout, neq
        if nout > 1 or neq > 1:
            to = self._keep(np.array([int(getattr(t, "out", 0)) for t in terms], dtype=np.int32))
            te = self._keep(np.array([int(getattr(t, "eq", 0)) for t in terms], dtype=np.int32))
            s.term_out = to.ctypes.data_as(C.POINTER(C.c_int))
            s.term_eq = te.ctypes.data_as(C.POINTER(C.c_int))
        if getattr(p, "out_scale", None) is not None:
            s.out_scale = self._keep(_arr(p.out_scale)).ctypes.data_as(_dp)
        groups = list(p.groups)
        s.ngroup = len(groups)
        ga = (PointGroup * max(1, len(groups)))()
        for k, g in enumerate(groups):
            for i in range(min(d, len(g.axes))):
                ax = self._keep(_arr(g.axes[i]))
                ga[k].n[i] = len(ax)
                ga[k].axis[i] = ax.ctypes.data_as(_dp)
                ga[k].deriv[i] = int(g.deriv[i])
            ga[k].y = self._keep(_arr(g.y).ravel()).ctypes.data_as(_dp)
            ga[k].noise_var = float(g.noise_var)
            ga[k].output = int(getattr(g, "out", 0))
            pts = getattr(g, "terms", None)
            if pts:
                ta = (PointTerm * len(pts))()
                for c, t in enumerate(pts):
                    for i in range(min(d, len(t.deriv))):
                        ta[c].deriv[i] = int(t.deriv[i])
                        if t.weights is not None and t.weights[i] is not None:
                            ta[c].weight[i] = self._keep(_arr(t.weights[i])).ctypes.data_as(_dp)
                    ta[c].coef = float(t.coef)
                    ta[c].output = int(t.out)
                self.keep.append(ta)
                ga[k].nterm = len(pts)
                ga[k].terms = C.cast(ta, C.POINTER(PointTerm))
        self.keep.append(ga)
        s.groups = C.cast(ga, C.POINTER(PointGroup))
        self.s = s

    def _keep(self, a):
        self.keep.append(a)
        return a


def validate(p) -> None:
    m = _Marshal(p)
    _check(lib().gpfvm_validate(C.byref(m.s)))


def assemble(p, max_iter: int = 512, tile: int = TILE_FP32, stream=None, reuse_memory: bool = True) -> C.c_void_p:
    m = _Marshal(p)
    o = AssembleOpts(max_iter, tile, 1 if reuse_memory else 0)
    h = C.c_void_p()
    _check(lib().gpfvm_assemble(C.byref(m.s), C.byref(o), _stream(stream), C.byref(h)))
    return h


def get_info(h) -> dict:
    info = HandleInfo()
    _check(lib().gpfvm_get_info(h, C.byref(info)), h)
    return {k: getattr(info, k) for k, _ in HandleInfo._fields_}


def matvec(h, x, y, nrhs: int = 1, prec: int = PREC_FP64, stream=None) -> None:
    """y = G x for device tensors x, y of n * nrhs elements, both float64 or both float32."""
    import torch
    if x.dtype != y.dtype or x.dtype not in (torch.float64, torch.float32):
        raise ValueError("matvec: x and y must both be float64 or both float32")
    dt = DTYPE_F64 if x.dtype == torch.float64 else DTYPE_F32
    _check(lib().gpfvm_matvec(h, nrhs, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), dt, prec,
                              _stream(stream)), h)


def volume_matvec(h, x, y, nrhs: int = 1, prec: int = PREC_FP64, stream=None) -> None:
    """y = (L_V k L_V' + Sigma_V) x (volume block only)."""
    _check(lib().gpfvm_volume_matvec(h, nrhs, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), prec,
                                     _stream(stream)), h)


def volume_matvec_noalloc(h, x, y, nrhs: int = 1, stream=None) -> None:
    """volume_matvec in float64 with no device allocation (static device scratch)."""
    _check(lib().gpfvm_volume_matvec_noalloc(h, nrhs, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                             _stream(stream)), h)


def schur_matvec(h, x, y, nrhs: int = 1, prec: int = PREC_FP64, stream=None) -> None:
    """y = S x (volume system after exact conditioning on the points)."""
    _check(lib().gpfvm_schur_matvec(h, nrhs, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), prec,
                                    _stream(stream)), h)


def default_solve_opts() -> SolveOpts:
    o = SolveOpts()
    lib().gpfvm_default_solve_opts(C.byref(o))
    return o


def solve(h, prec: int = PREC_FP64, tol: float = 1e-8, max_iter: int = 512, resume: bool = False,
          tile: int = TILE_FP32, block: int = 32, max_outer: int = 1000, check_every: int = 8,
          reorth_passes: int = 2, replace_every: int = 25, stream=None, raise_on_noconv: bool = False,
          coarsen: Optional[Sequence[int]] = None, method: int = METHOD_ITERGP) -> dict:
    """Solve of the volume system.  method: METHOD_ITERGP (directions stored,
    combined variance) or METHOD_CG (plain CG, mean only).  prec PREC_MIXED:
    blocks of `block` low-precision iterations, each re-stabilised in float64
    (tile must be the handle's tile format).  coarsen: per-dimension factors
    of the coarse warm start (the coarse cells become the first directions;
    None or all 1: off)."""
    cf = list(coarsen) if coarsen is not None else []
    cf = (cf + [1, 1, 1])[:3]
    o = SolveOpts(prec, tol, max_iter, 1 if resume else 0, tile, block, max_outer, check_every,
                  reorth_passes, replace_every, (C.c_int * 3)(*cf), method)
    info = SolveInfo()
    rc = lib().gpfvm_solve(h, C.byref(o), C.byref(info), _stream(stream))
    if rc not in (OK, E_NOCONV, E_NOTPD) or (raise_on_noconv and rc != OK):
        _check(rc, h)
    out = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
    out["rc"] = rc
    return out


def posterior(h, axes: Sequence[np.ndarray], mean, var=None, stream=None) -> None:
    """Posterior mean (and combined variance) on the grid; for a system with
    nout outputs, mean and var hold nout * prod(len(a) for a in axes) values,
    output-major."""
    d = len(axes)
    ax = [_arr(a) for a in axes]
    n = (C.c_int * d)(*[len(a) for a in ax])
    ptrs = (_dp * d)(*[a.ctypes.data_as(_dp) for a in ax])
    _check(lib().gpfvm_posterior(h, d, n, ptrs, C.c_void_p(mean.data_ptr()),
                                 C.c_void_p(var.data_ptr()) if var is not None else None, _stream(stream)), h)


def refine_variance(h, axes: Sequence[np.ndarray], weights, stream=None) -> dict:
    """Targeted uncertainty reduction: one extra IterGP iteration per row of
    `weights` (iters x prod(len(a) for a in axes)), the action of row i being
    the residual of K_S(grid) weights[i]."""
    d = len(axes)
    ax = [_arr(a) for a in axes]
    n = (C.c_int * d)(*[len(a) for a in ax])
    ptrs = (_dp * d)(*[a.ctypes.data_as(_dp) for a in ax])
    w = np.ascontiguousarray(weights, dtype=np.float64)
    if w.ndim != 2 or w.shape[1] != int(np.prod([len(a) for a in ax])):
        raise ValueError("weights must be a 2-D array (iterations x grid points)")
    info = SolveInfo()
    rc = lib().gpfvm_refine_variance(h, d, n, ptrs, int(w.shape[0]), w.ctypes.data_as(_dp), C.byref(info),
                                     _stream(stream))
    if rc not in (OK, E_NOTPD):
        _check(rc, h)
    out = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
    out["rc"] = rc
    return out


def weights(h, out, stream=None) -> None:
    _check(lib().gpfvm_weights(h, C.c_void_p(out.data_ptr()), _stream(stream)), h)


def gram_block(h, r0: int, nr: int, c0: int, nc: int, out, ld: Optional[int] = None, stream=None) -> None:
    _check(lib().gpfvm_gram_block(h, r0, nr, c0, nc, C.c_void_p(out.data_ptr()), ld or nc, _stream(stream)), h)


KERNEL_SE, KERNEL_MATERN12, KERNEL_MATERN32, KERNEL_MATERN52, KERNEL_MATERN72 = 0, 1, 2, 3, 4


def factor(kind: int, p: int, q: int, a1, a2, lengthscale: float, out, stream=None, kernel: int = KERNEL_SE) -> None:
    a1 = _arr(a1); a2 = _arr(a2)
    n1 = len(a1) - 1 if kind == 0 else len(a1)
    n2 = len(a2) if kind == 2 else len(a2) - 1
    _check(lib().gpfvm_factor(kind, kernel, p, q, n1, a1.ctypes.data_as(_dp), n2, a2.ctypes.data_as(_dp),
                              float(lengthscale), C.c_void_p(out.data_ptr()), _stream(stream)))


def destroy(h) -> None:
    if h:
        lib().gpfvm_destroy(h)


@dataclass
class Solved:
    """Convenience: one IBVP assembled, solved and evaluated on its grid."""
    mean: "object"
    var: "object"
    info: dict


def solve_ibvp(p, prec: int = PREC_FP64, tol: float = 1e-8, max_iter: int = 512, grid=None, with_var=True,
               device: str = "cuda:0", **kw) -> Solved:
    import torch
    h = assemble(p, max_iter=max_iter)
    try:
        info = solve(h, prec=prec, tol=tol, max_iter=max_iter, **kw)
        axes = grid if grid is not None else p.grid
        M = int(np.prod([len(a) for a in axes]))
        mean = torch.empty(M, dtype=torch.float64, device=device)
        var = torch.empty(M, dtype=torch.float64, device=device) if with_var else None
        posterior(h, axes, mean, var)
        torch.cuda.synchronize()
        return Solved(mean, var, info)
    finally:
        destroy(h)


# ---------------------------------------------------------------------------
# continuous-batching server
# ---------------------------------------------------------------------------
class Server:
    """Thin wrapper over gpfvm_server_*: submit whole IBVP solves, poll results."""

    def __init__(self, workers: int = 8, hbm_budget: int = 64 << 30, prec: int = PREC_FP64, tol: float = 1e-6,
                 max_iter: int = 1024, check_every: int = 16, coarse_cells: int = 0, max_batch: int = 16):
        o = ServerOpts(workers, hbm_budget, prec, tol, max_iter, check_every, coarse_cells, max_batch)
        self.h = C.c_void_p()
        _check(lib().gpfvm_server_create(C.byref(o), C.byref(self.h)))
        self.grids = {}

    def submit(self, p, grid=None) -> int:
        m = _Marshal(p)
        axes = [_arr(a) for a in (grid if grid is not None else p.grid)]
        d = len(axes)
        n = (C.c_int * d)(*[len(a) for a in axes])
        ptrs = (_dp * d)(*[a.ctypes.data_as(_dp) for a in axes])
        t = C.c_longlong()
        _check(lib().gpfvm_server_submit(self.h, C.byref(m.s), d, n, ptrs, C.byref(t)))
        self.grids[t.value] = int(np.prod([len(a) for a in axes]))
        return t.value

    def poll(self, ticket: int, wait: bool = False):
        """(done, result-dict or None, mean, var) with host numpy arrays."""
        M = self.grids[ticket]
        done = C.c_int()
        res = RequestResult()
        mean = np.empty(M)
        var = np.empty(M)
        _check(lib().gpfvm_server_poll(self.h, ticket, 1 if wait else 0, C.byref(done), C.byref(res),
                                       mean.ctypes.data_as(_dp), var.ctypes.data_as(_dp)))
        if not done.value:
            return False, None, None, None
        r = {"rc": res.rc, "t_submit": res.t_submit, "t_start": res.t_start, "t_done": res.t_done,
             "est_bytes": res.est_bytes, "n_grid": res.n_grid, "batch": res.batch}
        r.update({k: getattr(res.info, k) for k, _ in SolveInfo._fields_})
        return True, r, mean, var

    def stats(self) -> dict:
        st = ServerInfo()
        _check(lib().gpfvm_server_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerInfo._fields_}

    def close(self):
        if self.h:
            lib().gpfvm_server_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
