"""MI355X (gfx950) accelerated cyclic reduction: thin Python binding.

Argument marshalling only: every step of setup, apply, Krylov and
gradient runs in ``libacr.so`` (HIP kernels behind the C ABI declared in
``include/acr.h``).  PyTorch provides device memory and streams.

Entry points mirror the C ABI: :func:`acr_setup`, :func:`acr_apply`,
:func:`acr_apply_T`, :func:`acr_matvec`, :func:`krylov_solve`,
:func:`acr_grad_kappa`, :func:`acr_stats`, :func:`acr_destroy`; plus the
convenience wrappers :class:`Preconditioner` and :class:`ACRSolve` (a
``torch.autograd.Function`` whose backward solves the adjoint system with
the transposed factors).
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libacr.so")

POISSON_HARMONIC, CONVDIFF_UPWIND, HELMHOLTZ, STENCIL7_RAW, CONVDIFF_RECIRC, HELMHOLTZ_FEM27 = 0, 1, 2, 3, 4, 5
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
CG, FCG, GMRES = 0, 1, 2
MAX_LEVELS = 32
STATUS = ["OK", "E_INVALID", "E_NUMERIC", "E_NOMEM", "E_SINGULAR", "E_BREAKDOWN", "E_NOTCONV", "E_DEVICE",
          "E_RANK"]


class AcrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS[status] if 0 <= status < len(STATUS) else status}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("kappa", ctypes.c_void_p), ("beta_amp", ctypes.c_double), ("beta_phase", ctypes.c_double),
                ("c", ctypes.c_void_p), ("omega", ctypes.c_double), ("stencil7", ctypes.c_void_p)]


_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("eta", ctypes.c_double), ("leaf_size", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("max_rank", ctypes.c_int32), ("dense_work", ctypes.c_int32),
                ("alloc", _ALLOC), ("free", _FREE), ("alloc_ctx", ctypes.c_void_p), ("flags", ctypes.c_uint64)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("relres_true", ctypes.c_double), ("status", ctypes.c_int32),
                ("variant", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("nplanes", ctypes.c_int32), ("plane_points", ctypes.c_int32),
                ("clusters", ctypes.c_int32), ("dense_leaves", ctypes.c_int32), ("lr_leaves", ctypes.c_int32),
                ("factors", ctypes.c_int32), ("retries", ctypes.c_int32), ("rank_overflow", ctypes.c_int32),
                ("max_rank", ctypes.c_int32 * MAX_LEVELS), ("mean_rank", ctypes.c_double * MAX_LEVELS),
                ("max_rank_all", ctypes.c_int32), ("bytes_factors", ctypes.c_double),
                ("bytes_allocated", ctypes.c_double), ("bytes_per_apply", ctypes.c_double),
                ("setup_seconds", ctypes.c_double), ("setup_flops", ctypes.c_double), ("precision", ctypes.c_int32),
                ("accum_launches", ctypes.c_int32), ("accum_seconds", ctypes.c_double),
                ("accum_flops", ctypes.c_double), ("dense_launches", ctypes.c_int32),
                ("dense_seconds", ctypes.c_double), ("dense_flops", ctypes.c_double),
                ("bytes_peak", ctypes.c_double), ("bytes_level", ctypes.c_double * MAX_LEVELS),
                ("level_seconds", ctypes.c_double * MAX_LEVELS), ("setup_flops_class", ctypes.c_double * 4),
                ("leaf_inverse_flops", ctypes.c_double), ("bytes_apply_image", ctypes.c_double),
                ("accum_bytes", ctypes.c_double), ("dense_bytes", ctypes.c_double)]

    def as_dict(self):
        lv = self.levels
        return {"levels": lv, "nplanes": self.nplanes, "plane_points": self.plane_points,
                "clusters": self.clusters, "dense_leaves": self.dense_leaves, "lr_leaves": self.lr_leaves,
                "factors": self.factors, "retries": self.retries, "rank_overflow": self.rank_overflow,
                "max_rank": list(self.max_rank[:lv]), "mean_rank": list(self.mean_rank[:lv]),
                "max_rank_all": self.max_rank_all, "bytes_factors": self.bytes_factors,
                "bytes_allocated": self.bytes_allocated, "bytes_per_apply": self.bytes_per_apply,
                "setup_seconds": self.setup_seconds, "setup_flops": self.setup_flops, "precision": self.precision,
                "accum_launches": self.accum_launches, "accum_seconds": self.accum_seconds,
                "accum_flops": self.accum_flops, "dense_launches": self.dense_launches,
                "dense_seconds": self.dense_seconds, "dense_flops": self.dense_flops,
                "bytes_peak": self.bytes_peak, "bytes_level": list(self.bytes_level[:lv]),
                "level_seconds": list(self.level_seconds[:lv]),
                "setup_flops_class": dict(zip(("products", "gram", "core", "rebuild"), self.setup_flops_class)),
                "leaf_inverse_flops": self.leaf_inverse_flops, "bytes_apply_image": self.bytes_apply_image,
                "accum_bytes": self.accum_bytes, "dense_bytes": self.dense_bytes}


class Factor(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("role", ctypes.c_int32), ("plane", ctypes.c_int32),
                ("diag", ctypes.c_int32), ("ranks", ctypes.c_void_p), ("data", ctypes.c_void_p)]


class FactorBlob(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("factors", ctypes.POINTER(Factor))]


FACTOR_DINV, FACTOR_A, FACTOR_C = 0, 1, 2


class GeometryInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("clusters", "leaf_clusters", "depth", "block_nodes", "leaves",
                                              "admissible", "dense_leaves", "lr_leaves")]


SYMBOLS = ["acr_setup", "acr_setup_batched", "acr_problem_offset", "acr_num_problems", "acr_apply", "acr_apply_T",
           "acr_matvec", "acr_get_stencil", "krylov_solve", "acr_grad_kappa", "acr_stats", "acr_destroy",
           "acr_status_string", "acr_last_error", "acr_default_options", "acr_plane_geometry",
           "acr_import_factors", "krylov_solve_static"]

_lib = None


def lib():
    """Load ``libacr.so``; raises if the HIP extension has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1712_08872_amd.build`")
    # torch ships its own HIP runtime (soname libamdhip64.so.7); loading it
    # first makes libacr bind to that same runtime instead of a second copy
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.acr_setup.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options), vp, ctypes.POINTER(vp)]
    L.acr_setup_batched.argtypes = [ctypes.POINTER(Problem), i32, ctypes.POINTER(Options), vp, ctypes.POINTER(vp)]
    p64 = ctypes.POINTER(ctypes.c_int64)
    L.acr_problem_offset.argtypes = [vp, i32, p64, p64, p64, p64]
    L.acr_num_problems.argtypes = [vp]
    L.acr_num_problems.restype = i32
    L.acr_apply.argtypes = [vp, vp, vp, i32, vp]
    L.acr_apply_T.argtypes = [vp, vp, vp, i32, vp]
    L.acr_matvec.argtypes = [vp, i32, vp, vp, vp]
    L.acr_get_stencil.argtypes = [vp, vp, vp]
    L.krylov_solve.argtypes = [vp, i32, i32, i32, dbl, i32, vp, vp, ctypes.POINTER(SolveInfo), vp]
    L.krylov_solve_static.argtypes = [vp, i32, i32, i32, dbl, i32, vp, vp, ctypes.POINTER(SolveInfo), vp]
    L.acr_grad_kappa.argtypes = [vp, vp, vp, vp, vp]
    L.acr_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.acr_destroy.argtypes = [vp]
    L.acr_destroy.restype = None
    L.acr_status_string.argtypes = [i32]
    L.acr_status_string.restype = ctypes.c_char_p
    L.acr_last_error.restype = ctypes.c_char_p
    L.acr_import_factors.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(FactorBlob),
                                     vp, ctypes.POINTER(vp)]
    L.acr_plane_geometry.argtypes = [i32, i32, ctypes.POINTER(Options), ctypes.POINTER(GeometryInfo), vp, vp, i32]
    L.acr_default_options.argtypes = [ctypes.POINTER(Options)]
    L.acr_default_options.restype = None
    for name in ["acr_setup", "acr_setup_batched", "acr_problem_offset", "acr_apply", "acr_apply_T", "acr_matvec",
                 "acr_get_stencil", "krylov_solve", "acr_grad_kappa", "acr_stats", "acr_plane_geometry", "acr_import_factors",
                 "krylov_solve_static"]:
        getattr(L, name).restype = i32
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise AcrError(st, lib().acr_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, n, name):
    """Refuse a tensor whose length differs from what the library will
    read or write through its pointer (a wrong size would be an
    out-of-bounds device access, which the C ABI cannot detect)."""
    if t is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")


def _grid(nx, ny, nz):
    return (nx + 2) * (ny + 2) * (nz + 2)


def _check_problem(nx, ny, nz, kappa, c, stencil7):
    if min(nx, ny, nz) >= 1:
        _need(kappa, _grid(nx, ny, nz), "kappa")
        _need(c, _grid(nx, ny, nz), "c")
        _need(stencil7, 7 * nx * ny * nz, "stencil7")


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def default_options(**kw):
    o = Options()
    lib().acr_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Handle:
    """Owns an ``acr_handle``; keeps the input tensors alive.  ``n`` is the
    grid of a single-problem handle; ``offsets`` lists (off, N, grid_off,
    grid_N) per problem; ``total``/``grid_total`` are the concatenated
    lengths."""

    def __init__(self, ptr, n, keep, kinds=None):
        self.ptr = ptr
        self.n = n
        self._keep = keep
        self.kinds = list(kinds) if kinds is not None else []
        L = lib()
        self.offsets = []
        for i in range(L.acr_num_problems(ptr)):
            a, b, c, d = (ctypes.c_int64() for _ in range(4))
            _check(L.acr_problem_offset(ptr, i, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
            self.offsets.append((a.value, b.value, c.value, d.value))
        self.total = sum(o[1] for o in self.offsets)
        self.grid_total = sum(o[3] for o in self.offsets)
        # stencil rows per unknown of each problem (27 for the finite-element operator)
        self.stencil_total = sum((27 if k == HELMHOLTZ_FEM27 else 7) * o[1]
                                 for k, o in zip(self.kinds or [POISSON_HARMONIC] * len(self.offsets), self.offsets))

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "ptr", None):
            try:
                lib().acr_destroy(self.ptr)
            except Exception:  # interpreter shutdown: module globals already cleared
                pass
            self.ptr = None


def acr_setup(nx, ny, nz, kind=POISSON_HARMONIC, kappa=None, beta_amp=0.0, beta_phase=0.0, c=None, omega=0.0,
              stencil7=None, eps=1e-4, eta=2.0, leaf_size=32, precision=FP64, max_rank=0, dense_work=0,
              stream=None):
    """``acr_setup``: returns a :class:`Handle`.  Tensors are float64 CUDA."""
    _check_problem(nx, ny, nz, kappa, c, stencil7)
    p = Problem(nx, ny, nz, kind, _ptr(kappa), beta_amp, beta_phase, _ptr(c), omega, _ptr(stencil7))
    o = default_options(eps=eps, eta=eta, leaf_size=leaf_size, precision=precision, max_rank=max_rank,
                        dense_work=dense_work)
    out = ctypes.c_void_p()
    _check(lib().acr_setup(ctypes.byref(p), ctypes.byref(o), _stream(stream), ctypes.byref(out)))
    return Handle(out, (nx, ny, nz), (kappa, c, stencil7), [kind])


def acr_setup_batched(problems, eps=1e-4, eta=2.0, leaf_size=32, precision=FP64, max_rank=0, dense_work=0,
                      stream=None):
    """``acr_setup_batched``: ``problems`` is a list of dicts with the keys of
    :func:`acr_setup` (nx, ny, nz, kind, kappa, beta_amp, beta_phase, c,
    omega, stencil7).  Returns one :class:`Handle`."""
    arr = (Problem * len(problems))()
    keep = []
    for d in problems:
        _check_problem(d["nx"], d["ny"], d["nz"], d.get("kappa"), d.get("c"), d.get("stencil7"))
    for i, d in enumerate(problems):
        arr[i] = Problem(d["nx"], d["ny"], d["nz"], d.get("kind", POISSON_HARMONIC), _ptr(d.get("kappa")),
                         d.get("beta_amp", 0.0), d.get("beta_phase", 0.0), _ptr(d.get("c")), d.get("omega", 0.0),
                         _ptr(d.get("stencil7")))
        keep.append((d.get("kappa"), d.get("c"), d.get("stencil7")))
    o = default_options(eps=eps, eta=eta, leaf_size=leaf_size, precision=precision, max_rank=max_rank,
                        dense_work=dense_work)
    out = ctypes.c_void_p()
    _check(lib().acr_setup_batched(arr, len(problems), ctypes.byref(o), _stream(stream), ctypes.byref(out)))
    return Handle(out, None, keep, [d.get("kind", POISSON_HARMONIC) for d in problems])


def _nrhs(h, r, z):
    if r.numel() == 0 or r.numel() % h.total:
        raise ValueError(f"r has {r.numel()} elements, not a positive multiple of the handle's {h.total} unknowns")
    _need(z, r.numel(), "z")
    return r.numel() // h.total


def acr_apply(h, r, z=None, stream=None):
    import torch
    z = torch.empty_like(r) if z is None else z
    nrhs = _nrhs(h, r, z)
    _check(lib().acr_apply(h.ptr, _ptr(r), _ptr(z), nrhs, _stream(stream)))
    return z


def acr_apply_T(h, r, z=None, stream=None):
    import torch
    z = torch.empty_like(r) if z is None else z
    nrhs = _nrhs(h, r, z)
    _check(lib().acr_apply_T(h.ptr, _ptr(r), _ptr(z), nrhs, _stream(stream)))
    return z


def acr_matvec(h, x, transpose=False, y=None, stream=None):
    import torch
    y = torch.empty_like(x) if y is None else y
    _need(x, h.total, "x")
    _need(y, h.total, "y")
    _check(lib().acr_matvec(h.ptr, int(transpose), _ptr(x), _ptr(y), _stream(stream)))
    return y


def acr_get_stencil(h, stream=None):
    import torch
    out = torch.empty(h.stencil_total, dtype=torch.float64, device="cuda")
    _check(lib().acr_get_stencil(h.ptr, _ptr(out), _stream(stream)))
    return out


def krylov_solve(h, b, x=None, method=CG, restart=30, transpose=False, rtol=1e-8, maxit=1000, stream=None,
                 raise_on_fail=True, static_workspace=False):
    """Returns ``(x, info_dict)``.  ``static_workspace=True`` calls
    ``krylov_solve_static`` (the work vectors in the library's fixed device
    array; no allocation by the library)."""
    import torch
    x = torch.zeros_like(b) if x is None else x
    _need(b, h.total, "b")
    _need(x, h.total, "x")
    info = SolveInfo()
    fn = lib().krylov_solve_static if static_workspace else lib().krylov_solve
    st = fn(h.ptr, method, restart, int(transpose), rtol, maxit, _ptr(b), _ptr(x),
                            ctypes.byref(info), _stream(stream))
    d = {"iters": info.iters, "relres_true": info.relres_true, "status": info.status, "variant": info.variant}
    if st != 0 and raise_on_fail:
        _check(st)
    d["status"] = st
    return x, d


def acr_grad_kappa(h, u, lam, out=None, stream=None):
    import torch
    _need(u, h.total, "u")
    _need(lam, h.total, "lam")
    out = torch.empty(h.grid_total, dtype=torch.float64, device="cuda") if out is None else out
    _need(out, h.grid_total, "out")
    _check(lib().acr_grad_kappa(h.ptr, _ptr(u), _ptr(lam), _ptr(out), _stream(stream)))
    return out


def acr_stats(h):
    s = Stats()
    _check(lib().acr_stats(h.ptr, ctypes.byref(s)))
    return s.as_dict()


def acr_import_factors(nx, ny, nz, factors, kind=POISSON_HARMONIC, kappa=None, beta_amp=0.0, beta_phase=0.0,
                       c=None, omega=0.0, stencil7=None, eps=1e-4, eta=2.0, leaf_size=32, precision=FP64,
                       dense_work=0, stream=None):
    """``acr_import_factors``: a :class:`Handle` whose preconditioner is the
    given factorisation.  ``factors`` is a list of dicts with keys level,
    role (FACTOR_DINV / FACTOR_A / FACTOR_C), plane, diag (bool), ranks
    (int32 numpy array, one per leaf; H-matrix factors) and data (float64
    numpy array: the leaves in the order of :func:`acr_plane_geometry`, or
    the diagonal), all on the host."""
    import numpy as np
    _check_problem(nx, ny, nz, kappa, c, stencil7)
    keep = []
    arr = (Factor * len(factors))()
    for i, f in enumerate(factors):
        data = np.ascontiguousarray(f["data"], dtype=np.float64)
        ranks = None if f.get("diag") else np.ascontiguousarray(f["ranks"], dtype=np.int32)
        keep.append((data, ranks))
        arr[i] = Factor(f["level"], f["role"], f["plane"], int(bool(f.get("diag"))),
                        None if ranks is None else ranks.ctypes.data_as(ctypes.c_void_p),
                        data.ctypes.data_as(ctypes.c_void_p))
    blob = FactorBlob(len(factors), arr)
    p = Problem(nx, ny, nz, kind, _ptr(kappa), beta_amp, beta_phase, _ptr(c), omega, _ptr(stencil7))
    o = default_options(eps=eps, eta=eta, leaf_size=leaf_size, precision=precision, dense_work=dense_work)
    out = ctypes.c_void_p()
    _check(lib().acr_import_factors(ctypes.byref(p), ctypes.byref(o), ctypes.byref(blob), _stream(stream),
                                    ctypes.byref(out)))
    return Handle(out, (nx, ny, nz), (kappa, c, stencil7), [kind])


def acr_plane_geometry(nx, ny, eta=2.0, leaf_size=32, dense_work=0, eps=1e-4):
    """``acr_plane_geometry`` (host only): returns ``(info, perm, leaves)``
    with ``info`` a dict of counts, ``perm`` the H-order permutation
    (int32 numpy array of nx*ny) and ``leaves`` an (nleaves, 6) int32 array
    of (r0, c0, m, n, admissible, low_rank) in the library's leaf order."""
    import numpy as np
    o = default_options(eps=eps, eta=eta, leaf_size=leaf_size, dense_work=dense_work)
    info = GeometryInfo()
    _check(lib().acr_plane_geometry(nx, ny, ctypes.byref(o), ctypes.byref(info), None, None, 0))
    perm = np.empty(nx * ny, dtype=np.int32)
    leaves = np.empty((info.leaves, 6), dtype=np.int32)
    _check(lib().acr_plane_geometry(nx, ny, ctypes.byref(o), ctypes.byref(info), perm.ctypes.data_as(ctypes.c_void_p),
                                    leaves.ctypes.data_as(ctypes.c_void_p), info.leaves))
    return {k: getattr(info, k) for k, _ in GeometryInfo._fields_}, perm, leaves


def acr_destroy(h):
    h.close()


class Preconditioner:
    """ACR preconditioner of one problem (wraps a handle)."""

    def __init__(self, nx, ny, nz, **kw):
        self.h = acr_setup(nx, ny, nz, **kw)

    def apply(self, r):
        return acr_apply(self.h, r)

    def apply_T(self, r):
        return acr_apply_T(self.h, r)

    def solve(self, b, **kw):
        return krylov_solve(self.h, b, **kw)

    def stats(self):
        return acr_stats(self.h)


def _make_autograd():
    import torch

    class ACRSolve(torch.autograd.Function):
        """``u = A(kappa)^{-1} f`` for the harmonic-average Poisson operator.

        forward: ACR setup + preconditioned CG.  backward: the adjoint
        ``A^T lam = grad_u`` solved with CG preconditioned by the transposed
        factors (``acr_apply_T``), then ``dJ/dkappa = -lam^T (dA/dkappa) u``
        by the gradient stencil kernel; ``dJ/df = lam``.
        """

        @staticmethod
        def forward(ctx, kappa, f, n, eps=1e-4, eta=2.0, precision=FP64, rtol=1e-10, maxit=500):
            nx, ny, nz = n
            kap = kappa.detach().contiguous()
            h = acr_setup(nx, ny, nz, POISSON_HARMONIC, kappa=kap, eps=eps, eta=eta, precision=precision)
            u, info = krylov_solve(h, f.detach().contiguous(), method=CG, rtol=rtol, maxit=maxit)
            ctx.h = h
            ctx.rtol, ctx.maxit = rtol, maxit
            ctx.save_for_backward(u)
            ctx.info = info
            return u

        @staticmethod
        def backward(ctx, gu):
            (u,) = ctx.saved_tensors
            lam, _ = krylov_solve(ctx.h, gu.contiguous(), method=CG, transpose=True, rtol=ctx.rtol,
                                  maxit=ctx.maxit)
            gk = acr_grad_kappa(ctx.h, u, lam)
            return gk, lam, None, None, None, None, None, None

    return ACRSolve


def __getattr__(name):
    if name == "ACRSolve":
        cls = _make_autograd()
        globals()["ACRSolve"] = cls
        return cls
    raise AttributeError(name)
