"""ctypes binding of libbkwd.so (include/bkwd.h).

Argument marshalling only: every operation runs in the HIP library.  Device
memory comes from PyTorch; the stream is torch's current stream.  There is no
fallback: if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbkwd.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EBREAKDOWN = 0, -1, -2, -3, -4, -5
FP64, FP32, MIXED = 0, 1, 2
BICGSTAB, BLOCK_BICGSTAB, BLOCK_BICGGR = 0, 1, 2
COMPRESS12 = 1
SITE_MAJOR, COMPONENT_MAJOR = 0, 1
LAYOUTS = {"site": SITE_MAJOR, "component": COMPONENT_MAJOR}
MAX_RHS = 64

METHODS = {"bicgstab": BICGSTAB, "block_bicgstab": BLOCK_BICGSTAB, "block_bicggr": BLOCK_BICGGR}
PRECS = {"fp64": FP64, "fp32": FP32, "mixed": MIXED}


class BkwdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bkwd error {code}: {msg}")
        self.code = code


class NotConverged(RuntimeError):
    """ENOCONV or EBREAKDOWN: the solve stopped; ``info`` and the last iterate
    are attached."""

    def __init__(self, code: int, msg: str, info: dict, X):
        super().__init__(f"bkwd solve status {code}: {msg} (info={info})")
        self.code = code
        self.info = info
        self.X = X


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("max_restarts", ctypes.c_int),
        ("use_x0", ctypes.c_int),
        ("shadow", ctypes.c_int),
        ("check_every", ctypes.c_int),
        ("stagnation", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
        ("seed", ctypes.c_ulonglong),
        ("history", ctypes.POINTER(ctypes.c_double)),
        ("history_len", ctypes.c_int),
        ("profile", ctypes.c_int),
        ("shadow_block", ctypes.c_void_p),
        ("qr_frame", ctypes.c_int),
        ("dagger", ctypes.c_int),
        ("reliable", ctypes.c_double),
        ("max_block", ctypes.c_int),
        ("evenodd", ctypes.c_int),
        ("deflate", ctypes.c_int),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("outer_cycles", ctypes.c_int),
        ("matvecs", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("status_detail", ctypes.c_int),
        ("history_written", ctypes.c_int),
        ("true_residual_max", ctypes.c_double),
        ("recursive_residual_max", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("dslash_ms", ctypes.c_double),
        ("dslash_calls", ctypes.c_int),
        ("dslash_calls_fp32", ctypes.c_int),
        ("dslash_ms_fp32", ctypes.c_double),
        ("update_ms", ctypes.c_double * 3),
        ("update_calls", ctypes.c_int * 3),
        ("reliable_updates", ctypes.c_int),
        ("main_width", ctypes.c_int),
        ("dslash_ms_fp32_main", ctypes.c_double),
        ("dslash_calls_fp32_main", ctypes.c_int),
        ("update_ms_main", ctypes.c_double * 3),
        ("update_calls_main", ctypes.c_int * 3),
        ("deflated_columns", ctypes.c_int),
        ("gram_operator", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if isinstance(v, ctypes.Array) else v
        return d


_lib = None

# name -> (restype, argtypes); every function of include/bkwd.h
SIGNATURES = {
    "bkwd_lattice_bytes": (ctypes.c_size_t, [ctypes.POINTER(ctypes.c_int), ctypes.c_uint]),
    "bkwd_lattice_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), ctypes.c_void_p, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_uint, ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "bkwd_lattice_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]),
    "bkwd_lattice_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "bkwd_lattice_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
    "bkwd_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "bkwd_apply_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "bkwd_solve_opts_default": (None, [ctypes.POINTER(SolveOpts)]),
    "bkwd_solve_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(SolveOpts)]),
    "bkwd_block_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(SolveOpts), ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.POINTER(SolveInfo), ctypes.c_void_p]),
    "bkwd_true_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p]),
    "bkwd_true_residual_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "bkwd_meson_correlators": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "bkwd_gradients_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int]),
    "bkwd_gradients": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "bkwd_last_error": (ctypes.c_char_p, []),
    "bkwd_version": (ctypes.c_char_p, []),
}


def lib():
    """Load libbkwd.so once; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_0903_4936_amd.build.build()")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def last_error() -> str:
    return lib().bkwd_last_error().decode()


def _check(code: int):
    if code != OK:
        raise BkwdError(code, last_error())


def _dims_arr(dims):
    return (ctypes.c_int * 4)(*[int(d) for d in dims])


def lattice_bytes(dims, flags: int = 0) -> int:
    return int(lib().bkwd_lattice_bytes(_dims_arr(dims), flags))


def default_opts() -> SolveOpts:
    o = SolveOpts()
    lib().bkwd_solve_opts_default(ctypes.byref(o))
    return o


def _torch():
    import torch
    return torch


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _prec_of(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex128:
        return FP64
    if t.dtype == torch.complex64:
        return FP32
    raise ValueError("spinor blocks must be complex128 or complex64")


class Lattice:
    """D_W of Eq. (1) on the device for links U (numpy complex128,
    shape (4, Lt, Lz, Ly, Lx, 3, 3)), kappa and csw."""

    def __init__(self, links: np.ndarray, kappa: float, csw: float, flags: int = 0, device: str = "cuda"):
        torch = _torch()
        links = np.ascontiguousarray(links, dtype=np.complex128)
        if links.ndim != 7 or links.shape[0] != 4 or links.shape[-2:] != (3, 3):
            raise ValueError("links must have shape (4, Lt, Lz, Ly, Lx, 3, 3)")
        lt, lz, ly, lx = links.shape[1:5]
        self.dims = (lx, ly, lz, lt)
        self.volume = lx * ly * lz * lt
        self.device = torch.device(device)
        nbytes = lattice_bytes(self.dims, flags)
        if nbytes == 0:
            raise ValueError("invalid lattice dims")
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._buf.data_ptr()
        self._base = (base + 255) // 256 * 256
        self._nbytes = nbytes
        h = ctypes.c_void_p()
        code = lib().bkwd_lattice_create(_dims_arr(self.dims), links.ctypes.data_as(ctypes.c_void_p), float(kappa),
                                         float(csw), flags, ctypes.c_void_p(self._base), nbytes,
                                         _stream_ptr(self.device), ctypes.byref(h))
        _check(code)
        self._h = h
        self.kappa, self.csw, self.flags = float(kappa), float(csw), flags
        self._ws = None

    # ------------------------------------------------------------- lifetime
    def close(self):
        if getattr(self, "_h", None):
            lib().bkwd_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, kappa: float, csw: float):
        _check(lib().bkwd_lattice_set_params(self._h, float(kappa), float(csw), _stream_ptr(self.device)))
        self.kappa, self.csw = float(kappa), float(csw)

    # ------------------------------------------------------------- helpers
    def _as_block(self, X):
        torch = _torch()
        if not isinstance(X, torch.Tensor) or X.device.type != "cuda":
            raise ValueError("spinor blocks must be CUDA tensors")
        if not X.is_contiguous():
            raise ValueError("spinor blocks must be contiguous")
        L = X.shape[-1]
        if X.numel() != 12 * self.volume * L:
            raise ValueError(f"block has {X.numel()} elements, expected 12*V*L with L = {L}")
        if L < 1 or L > MAX_RHS:
            raise ValueError(f"L must be in 1..{MAX_RHS}")
        return L

    def _workspace(self, nbytes: int):
        torch = _torch()
        if self._ws is None or self._ws.numel() < nbytes + 256:
            self._ws = None
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        return (base + 255) // 256 * 256

    # ------------------------------------------------------------- operator
    def apply(self, X, dagger: bool = False, out=None, layout: str = "site"):
        """Y = D_W X (or D_W^dagger X) for every column of X.  ``layout``:
        "site" (X of shape (..., 4, 3, L), bkwd_apply) or "component" (the
        solver's Krylov layout [4][3][V][L], bkwd_apply_layout)."""
        torch = _torch()
        L = self._as_block(X)
        prec = _prec_of(X)
        Y = torch.empty_like(X) if out is None else out
        if Y.shape != X.shape or Y.dtype != X.dtype or not Y.is_contiguous():
            raise ValueError("out must match X")
        _check(lib().bkwd_apply_layout(self._h, int(bool(dagger)), L, prec, LAYOUTS[layout],
                                       ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                       _stream_ptr(self.device)))
        return Y

    # ------------------------------------------------------------- solves
    def make_opts(self, method="block_bicggr", prec="mixed", tol=1e-12, inner_tol=0.0, max_iter=10000,
                  max_restarts=20, shadow=0, seed=12345, check_every=8, stagnation=200, profile=False,
                  shadow_block=None, qr_frame=-1, dagger=False, reliable=None, max_block=0, evenodd=False,
                  deflate=False):
        o = default_opts()
        o.method = METHODS[method] if isinstance(method, str) else int(method)
        o.prec = PRECS[prec] if isinstance(prec, str) else int(prec)
        o.tol = float(tol)
        o.inner_tol = float(inner_tol)
        o.max_iter = int(max_iter)
        o.max_restarts = int(max_restarts)
        o.shadow = int(shadow)
        o.seed = int(seed)
        o.check_every = int(check_every)
        o.stagnation = int(stagnation)
        o.profile = int(bool(profile))
        o.qr_frame = int(qr_frame)
        o.dagger = int(bool(dagger))
        o.max_block = int(max_block)
        o.evenodd = int(bool(evenodd))
        o.deflate = int(bool(deflate))
        if reliable is not None:
            o.reliable = float(reliable)
        if shadow_block is not None:
            o.shadow = 2
            o.shadow_block = ctypes.c_void_p(shadow_block.data_ptr())
            self._shadow_ref = shadow_block
        return o

    def workspace_bytes(self, L: int, opts: SolveOpts) -> int:
        return int(lib().bkwd_solve_workspace_bytes(self._h, int(L), ctypes.byref(opts)))

    def block_solve(self, B, X=None, opts: SolveOpts = None, history_len: int = 0, raise_on_fail: bool = True,
                    **kw):
        """Solve D_W X = B (complex128 device blocks).  Returns (X, info)."""
        torch = _torch()
        L = self._as_block(B)
        if B.dtype != torch.complex128:
            raise ValueError("B must be complex128")
        if opts is None:
            opts = self.make_opts(**kw)
        elif kw:
            raise ValueError("pass either opts or keyword options")
        if X is None:
            X = torch.zeros_like(B)
            opts.use_x0 = 0
        elif X.shape != B.shape or X.dtype != B.dtype or not X.is_contiguous():
            raise ValueError("X must match B")
        else:
            opts.use_x0 = 1
        if opts.shadow == 2:
            sb = getattr(self, "_shadow_ref", None)
            if sb is None or sb.shape != B.shape or sb.dtype != B.dtype or not sb.is_contiguous():
                raise ValueError("shadow_block must match B")
        hist = None
        if history_len > 0:
            hist = (ctypes.c_double * history_len)()
            opts.history = hist
            opts.history_len = history_len
        nbytes = self.workspace_bytes(L, opts)
        if nbytes == 0:
            raise ValueError(last_error() or "invalid solve options")
        ws = self._workspace(nbytes)
        info = SolveInfo()
        code = lib().bkwd_block_solve(self._h, L, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                      ctypes.byref(opts), ctypes.c_void_p(ws), nbytes, ctypes.byref(info),
                                      _stream_ptr(self.device))
        d = info.as_dict()
        if hist is not None:
            d["history"] = list(hist[: info.history_written])
        if code in (ENOCONV, EBREAKDOWN):
            if raise_on_fail:
                raise NotConverged(code, last_error(), d, X)
            d["status"] = code
            return X, d
        _check(code)
        d["status"] = OK
        return X, d

    def true_residual(self, B, X) -> np.ndarray:
        """Per-column ||b_i - D x_i|| / ||b_i|| in FP64 (Sec. 4.3)."""
        L = self._as_block(B)
        opts = self.make_opts(method="block_bicggr", prec="fp64")
        nbytes = self.workspace_bytes(L, opts)
        ws = self._workspace(nbytes)
        out = (ctypes.c_double * L)()
        _check(lib().bkwd_true_residual(self._h, L, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                        out, ctypes.c_void_p(ws), nbytes, _stream_ptr(self.device)))
        return np.array(out[:L])

    def meson_correlators(self, X):
        """Pion and rho two-point functions (device float64 tensors of Lt
        values) from the 12 point-source solutions X (bkwd_meson_correlators)."""
        torch = _torch()
        L = self._as_block(X)
        if L != 12:
            raise ValueError("X must hold the 12 point-source solutions")
        if X.dtype != torch.complex128:
            raise ValueError("X must be complex128")
        lt = self.dims[3]
        pion = torch.empty(lt, dtype=torch.float64, device=X.device)
        rho = torch.empty(lt, dtype=torch.float64, device=X.device)
        _check(lib().bkwd_meson_correlators(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(pion.data_ptr()),
                                            ctypes.c_void_p(rho.data_ptr()), _stream_ptr(self.device)))
        return pion, rho

    # ------------------------------------------------------------- gradients
    def gradients(self, X, Lam, links: bool = True, scalars: bool = True) -> dict:
        """Given the solution X and the adjoint solution Lam = D^{-H} G of a
        loss with gradient G in X: {"kappa", "csw", "links"} (bkwd_gradients)."""
        torch = _torch()
        L = self._as_block(X)
        if Lam.shape != X.shape or X.dtype != torch.complex128 or Lam.dtype != torch.complex128:
            raise ValueError("X and Lam must be complex128 blocks of the same shape")
        if not Lam.is_contiguous():
            raise ValueError("Lam must be contiguous")
        nbytes = int(lib().bkwd_gradients_workspace_bytes(self._h, L))
        if nbytes == 0:
            raise ValueError(last_error() or "invalid arguments")
        ws = self._workspace(nbytes)
        gk, gc = ctypes.c_double(0.0), ctypes.c_double(0.0)
        lt, lz, ly, lx = self.dims[3], self.dims[2], self.dims[1], self.dims[0]
        gU = torch.empty((4, lt, lz, ly, lx, 3, 3), dtype=torch.complex128, device=self.device) if links else None
        _check(lib().bkwd_gradients(self._h, L, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Lam.data_ptr()),
                                    ctypes.byref(gk) if scalars else None, ctypes.byref(gc) if scalars else None,
                                    ctypes.c_void_p(gU.data_ptr()) if links else None, ctypes.c_void_p(ws), nbytes,
                                    _stream_ptr(self.device)))
        return {"kappa": gk.value if scalars else None, "csw": gc.value if scalars else None, "links": gU}
