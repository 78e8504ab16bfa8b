"""Python binding of libfd (filter-diagonalization hot path on MI355X / gfx950).

Argument marshalling only: every step of the computation runs in libfd's HIP
kernels and host code.  Device blocks are torch tensors on the GPU (2-D,
row-major, unit stride along the row); PyTorch provides memory and streams.
The library must be built (``python -m paper_2209_01974_amd.build`` or
``__graft_entry__.build()``); there is no fallback path.

Function names follow the C ABI in include/fd.h.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfd.so")

FD_OK, FD_ERR_INVALID, FD_ERR_OOM, FD_ERR_HIP, FD_ERR_NOT_CONVERGED, FD_ERR_BREAKDOWN, FD_ERR_UNSUPPORTED = range(7)
FD_F64, FD_F32 = 0, 1
FD_FMT_CSR, FD_FMT_SELL, FD_FMT_MATFREE, FD_FMT_PENCIL = 0, 1, 2, 3
FD_HUBBARD_RING, FD_ANDERSON_3D, FD_DIAGONAL, FD_USER_CSR = range(4)
FD_BUILD_HOST_ONLY = 1
FD_ORTHO_SVQB2, FD_ORTHO_CHOLQR2 = 0, 1

STATUS_NAMES = {0: "FD_OK", 1: "FD_ERR_INVALID", 2: "FD_ERR_OOM", 3: "FD_ERR_HIP",
                4: "FD_ERR_NOT_CONVERGED", 5: "FD_ERR_BREAKDOWN", 6: "FD_ERR_UNSUPPORTED"}


class FDError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status
        self.message = message


class ModelParams(C.Structure):
    _fields_ = [("model", C.c_int), ("L", C.c_int32), ("n_up", C.c_int32), ("n_dn", C.c_int32),
                ("periodic", C.c_int32), ("t", C.c_double), ("U", C.c_double), ("W", C.c_double),
                ("seed", C.c_uint64), ("n", C.c_int64), ("diag", C.c_void_p), ("D", C.c_int64),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p), ("skip", C.c_int64),
                ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("config_order", C.c_int32)]


class SolveParams(C.Structure):
    _fields_ = [("tau_lo", C.c_double), ("tau_hi", C.c_double), ("n_target", C.c_int32),
                ("n_search", C.c_int32), ("nb", C.c_int32), ("degree", C.c_int32),
                ("max_iter", C.c_int32), ("tol", C.c_double), ("precision", C.c_int32),
                ("ortho", C.c_int32), ("seed", C.c_uint64), ("adapt", C.c_int32), ("picker_dev", C.c_void_p),
                ("interval", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_conv", C.c_int32), ("iters_fp32", C.c_int32),
                ("spmmv_count", C.c_int64), ("t_filter", C.c_double), ("t_orthog", C.c_double),
                ("t_rr", C.c_double), ("t_total", C.c_double), ("norm_H", C.c_double),
                ("max_resid", C.c_double), ("degree", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_converged", C.c_int32), ("graph_launches", C.c_int64),
                ("t_filter", C.c_double), ("t_orthog", C.c_double), ("t_rr", C.c_double),
                ("t_total", C.c_double), ("nb", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_D = C.c_double

_SIGS = {
    "fd_build_matrix": [C.POINTER(ModelParams), C.c_int, _I32, _I32, _I32, C.POINTER(_P)],
    "fd_matrix_info": [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_D), C.POINTER(_D)],
    "fd_matrix_export_csr": [_P, _P, _P, _P],
    "fd_matrix_export_sell": [_P, _P, _P, _P, _P, _P],
    "fd_matrix_export_configs": [_P, _P, _P],
    "fd_lanczos": [_P, _I32, C.c_uint64, _P, _P, C.POINTER(_I32), _P],
    "fd_kpm_count": [_P, _I32, _I32, _I64, _D, _D, _P],
    "fd_debug_alloc_limit": [_I64],
    "fd_batch_autotune": [_P, C.c_int, _I32, _P, _P],
    "fd_spmmv": [_P, C.c_int, _I32, _P, _I64, _P, _I64, _P],
    "fd_cheb_filter": [_P, C.c_int, _I32, _I32, _P, _I64, _P, _I32, _D, _D, _P, _P, _I64, _P],
    "fd_cheb_coeffs": [_I32, _D, _D, _I32, _P],
    "fd_gram": [_I64, _I32, _I32, _P, _I64, _P, _I64, _P, _I64, _P],
    "fd_rotate": [_I64, _I32, _I32, _P, _I64, _P, _I64, _P],
    "fd_syev": [_I32, _P, _I64, _P, _P, _I64, _P],
    "fd_orthog": [_I64, _I32, _P, _I64, _I32, C.c_uint64, C.POINTER(_I32), _P],
    "fd_rayleigh_ritz": [_P, _I32, _I32, _P, _P, _I64, _P, _P, _P],
    "fd_solve": [_P, C.POINTER(SolveParams), _P, _P, _P, _P, C.POINTER(SolveStats)],
    "fd_spmmv_tune": [_I32, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _I32],
    "fd_stream": [_I32, _I64, _P, _P, _P, _D, _P],
    "fd_autotune": [_P, C.c_int, _I32, _P, _P],
    "fd_kpm_moments": [_P, _I32, _P, _I64, _I32, _D, _D, _P, _P, _I64, _P, _P],
    "fd_pick_degree": [_P, _D, _D, _I32, _I32, _P, C.c_uint64, C.POINTER(_I32), C.POINTER(_D), _P, _P],
    "fd_mlp_forward": [_P, _I32, _P, _P, _P],
    "fd_mlp_grad": [_P, _I32, _P, _P, _P, _P, _P, _P],
    "fd_mlp_adam": [_P, _P, _P, _P, _I32, C.c_float, C.c_float, _P],
    "fd_lehmann": [_I64, _I32, _P, _P, _I64, _D, _P, C.POINTER(_I32), _P, C.POINTER(_I32), _P],
    "fd_batch_create": [_I32, _P, C.POINTER(_P)],
    "fd_batch_info": [_P, C.POINTER(_I64), _P],
    "fd_batch_spmmv": [_P, C.c_int, _I32, _P, _I64, _P, _I64, _P],
    "fd_batch_filter": [_P, C.c_int, _I32, _I32, _P, _I64, _P, _P, _I32, _P, _P, _P, _P, _I64, _I32, _P],
    "fd_solve_batch": [_P, _P, _P, _P, _P, _P, _P, C.POINTER(BatchStats)],
}


def lib() -> C.CDLL:
    """Load libfd.so (raises if it has not been built: no fallback)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime; loading it first makes libfd bind
        # to that same runtime (one HIP runtime per process).
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfd.so not built at %s (run __graft_entry__.build())" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.fd_matrix_free.argtypes = [_P]
        L.fd_matrix_free.restype = None
        L.fd_batch_free.argtypes = [_P]
        L.fd_batch_free.restype = None
        L.fd_last_error.restype = C.c_char_p
        L.fd_syev_last_sweeps.restype = C.c_int32
        L.fd_syev_last_sweeps.argtypes = []
        _lib = L
    return _lib


def _check(st: int, allow=(FD_OK,)) -> int:
    if st not in allow:
        raise FDError(st, lib().fd_last_error().decode())
    return st


def _stream(stream) -> C.c_void_p:
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _blk(t, name: str):
    """(pointer, leading dimension, dtype code) of a 2-D row-major GPU tensor."""
    import torch
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("%s must be a 2-D tensor with unit column stride" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if t.dtype == torch.float64:
        dt = FD_F64
    elif t.dtype == torch.float32:
        dt = FD_F32
    else:
        raise ValueError("%s must be float64 or float32" % name)
    return C.c_void_p(t.data_ptr()), t.stride(0), dt


# --------------------------------------------------------------------- matrix --
class Matrix:
    """Owning wrapper of an fd_matrix handle."""

    def __init__(self, handle: C.c_void_p, fmt: int, C_: int):
        self._h = handle
        self.fmt = fmt
        self.C = C_
        D, nnz, stored = _I64(), _I64(), _I64()
        lo, hi = _D(), _D()
        _check(lib().fd_matrix_info(self._h, C.byref(D), C.byref(nnz), C.byref(stored),
                                    C.byref(lo), C.byref(hi)))
        self.D, self.nnz, self.stored = D.value, nnz.value, stored.value
        self.lam_lo, self.lam_hi = lo.value, hi.value

    @property
    def handle(self):
        return self._h

    def export_csr(self):
        rowptr = np.empty(self.D + 1, np.int64)
        col = np.empty(self.nnz, np.uint32)
        val = np.empty(self.nnz, np.float64)
        _check(lib().fd_matrix_export_csr(self._h, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data))
        return rowptr, col, val

    def export_sell(self):
        nch = (self.D + self.C - 1) // self.C
        perm = np.empty(self.D, np.int32)
        cptr = np.empty(nch + 1, np.int64)
        clen = np.empty(nch, np.int32)
        col = np.empty(self.stored, np.uint32)
        val = np.empty(self.stored, np.float64)
        _check(lib().fd_matrix_export_sell(self._h, perm.ctypes.data, cptr.ctypes.data, clen.ctypes.data,
                                           col.ctypes.data, val.ctypes.data))
        return perm, cptr, clen, col, val

    def export_configs(self, n_up_configs: int, n_dn_configs: int):
        """Spin configuration (bit mask) of every up and down label of a Hubbard matrix."""
        up = np.empty(n_up_configs, np.uint64)
        dn = np.empty(n_dn_configs, np.uint64)
        _check(lib().fd_matrix_export_configs(self._h, up.ctypes.data, dn.ctypes.data))
        return up, dn

    def free(self):
        if self._h:
            lib().fd_matrix_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_matrix(model: str, fmt: str = "csr", C_: int = 1, sigma: int = 1, host_only: bool = False,
                 L: int = 0, n_up: int = 0, n_dn: int = 0, periodic: bool = True, t: float = 1.0,
                 U: float = 0.0, W: float = 0.0, seed: int = 0, diag=None, csr=None, skip: int = 0,
                 tiles=(0, 0), config_order: int = 0) -> Matrix:
    """fd_build_matrix for model in {"hubbard", "anderson", "diagonal", "csr"} and fmt in
    {"csr", "sell", "matfree", "pencil"} ("matfree": Hubbard only, C_ = default up-pass tile;
    "pencil": Anderson only, C_ x sigma = (x, y) tile of the walk).  tiles = (tile_x, tile_y):
    Anderson sites numbered along the tile walk ((0, 0): natural numbering)."""
    p = ModelParams()
    keep = []
    codes = {"hubbard": FD_HUBBARD_RING, "anderson": FD_ANDERSON_3D, "diagonal": FD_DIAGONAL, "csr": FD_USER_CSR}
    p.model = codes[model]
    p.L, p.n_up, p.n_dn, p.periodic = L, n_up, n_dn, int(periodic)
    p.t, p.U, p.W, p.seed, p.skip = t, U, W, seed, skip
    p.tile_x, p.tile_y = int(tiles[0]), int(tiles[1])
    p.config_order = int(config_order)
    if diag is not None:
        d = np.ascontiguousarray(diag, dtype=np.float64)
        keep.append(d)
        p.n = d.size
        p.diag = d.ctypes.data
    if csr is not None:
        rowptr, col, val = (np.ascontiguousarray(csr[0], np.int64), np.ascontiguousarray(csr[1], np.uint32),
                            np.ascontiguousarray(csr[2], np.float64))
        keep += [rowptr, col, val]
        p.D = rowptr.size - 1
        p.rowptr, p.col, p.val = rowptr.ctypes.data, col.ctypes.data, val.ctypes.data
    f = {"csr": FD_FMT_CSR, "sell": FD_FMT_SELL, "matfree": FD_FMT_MATFREE, "pencil": FD_FMT_PENCIL}[fmt]
    h = C.c_void_p()
    _check(lib().fd_build_matrix(C.byref(p), f, C_, sigma, FD_BUILD_HOST_ONLY if host_only else 0, C.byref(h)))
    return Matrix(h, f, C_ if f == FD_FMT_SELL else 1)


# -------------------------------------------------------------------- kernels --
def spmmv(m: Matrix, X, Y, stream=None) -> None:
    """Y = A X (fd_spmmv); nb = X.shape[1]."""
    px, ldx, dt = _blk(X, "X")
    py, ldy, dty = _blk(Y, "Y")
    if dt != dty or X.shape != Y.shape or X.shape[0] != m.D:
        raise ValueError("X and Y must be D x nb blocks of one dtype")
    _check(lib().fd_spmmv(m.handle, dt, X.shape[1], px, ldx, py, ldy, _stream(stream)))


def cheb_filter(m: Matrix, V, mu, alpha: float, beta: float, W1, W2, nb: int, stream=None) -> None:
    """V <- p[alpha A + beta] V bundle by bundle (fd_cheb_filter)."""
    pv, ldv, dt = _blk(V, "V")
    p1, ldw, d1 = _blk(W1, "W1")
    p2, ldw2, d2 = _blk(W2, "W2")
    if not (dt == d1 == d2) or ldw != ldw2:
        raise ValueError("V, W1, W2 must share a dtype and W1, W2 a leading dimension")
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    if V.shape[1] % nb:
        raise ValueError("V width must be a multiple of nb")
    _check(lib().fd_cheb_filter(m.handle, dt, nb, V.shape[1] // nb, pv, ldv, mu.ctypes.data, mu.size - 1,
                                alpha, beta, p1, p2, ldw, _stream(stream)))


def cheb_coeffs(kind: int, a: float, b: float, degree: int) -> np.ndarray:
    mu = np.empty(degree + 1)
    _check(lib().fd_cheb_coeffs(kind, a, b, degree, mu.ctypes.data))
    return mu


def gram(X, Y, G, stream=None) -> None:
    """G = X^t Y (fd_gram), FP64."""
    px, ldx, _ = _blk(X, "X")
    py, ldy, _ = _blk(Y, "Y")
    pg, ldg, _ = _blk(G, "G")
    _check(lib().fd_gram(X.shape[0], X.shape[1], Y.shape[1], px, ldx, py, ldy, pg, ldg, _stream(stream)))


def rotate(X, Q, stream=None) -> None:
    """X[:, :n] <- X Q in place (fd_rotate), Q is m x n."""
    px, ldx, _ = _blk(X, "X")
    pq, ldq, _ = _blk(Q, "Q")
    _check(lib().fd_rotate(X.shape[0], Q.shape[0], Q.shape[1], px, ldx, pq, ldq, _stream(stream)))


def syev(S, w, U, stream=None) -> None:
    """S = U diag(w) U^t on the GPU (fd_syev); S is overwritten."""
    ps, lds, _ = _blk(S, "S")
    pu, ldu, _ = _blk(U, "U")
    _check(lib().fd_syev(S.shape[0], ps, lds, C.c_void_p(w.data_ptr()), pu, ldu, _stream(stream)))


def spmmv_tune(order: int = 0, xcd: int = 2, iters: int = 1, grid: int = 1024, nontemporal: int = 1,
               wide: int = 0, tile: int = 0, shfl: int = 2, lpr: int = 0, lds: int = 0) -> None:
    """Launch shape of the sparse kernels (process-wide; results unchanged,
    except lpr > 0 for one vector, which sums a row's entries in another
    order)."""
    _check(lib().fd_spmmv_tune(order, xcd, iters, grid, nontemporal, wide, tile, shfl, lpr, lds))


def kpm_moments(m: "Matrix", R, nmom: int, alpha: float, beta: float, stream=None) -> np.ndarray:
    """KPM moments mu_k = <r|T_k(alpha A + beta)|r> / D averaged over the
    columns r of the GPU block R (fd_kpm_moments)."""
    import torch
    pr, ldr, dt = _blk(R, "R")
    if dt != FD_F64:
        raise ValueError("R must be float64")
    w = min(R.shape[1], 64)
    W1 = torch.empty((R.shape[0], w), dtype=torch.float64, device=R.device)
    W2 = torch.empty_like(W1)
    mu = np.empty(nmom)
    _check(lib().fd_kpm_moments(m.handle, R.shape[1], pr, ldr, nmom, alpha, beta, C.c_void_p(W1.data_ptr()),
                                C.c_void_p(W2.data_ptr()), W1.stride(0), mu.ctypes.data, _stream(stream)))
    return mu


MLP_IN, MLP_HIDDEN, MLP_OUT = 66, 128, 2
MLP_NPARAMS = MLP_HIDDEN * MLP_IN + MLP_HIDDEN + 2 * (MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN) + MLP_OUT * MLP_HIDDEN + MLP_OUT


def pick_degree(m: "Matrix", tau_lo: float, tau_hi: float, n_target: int, n_search: int, picker=None,
                seed: int = 0):
    """(degree, first window half-width, network inputs) from fd_pick_degree."""
    deg = _I32()
    rad = _D()
    feat = np.empty(MLP_IN, np.float32)
    _check(lib().fd_pick_degree(m.handle, tau_lo, tau_hi, n_target, n_search,
                                C.c_void_p(picker.data_ptr()) if picker is not None else None, seed,
                                C.byref(deg), C.byref(rad), feat.ctypes.data, _stream(None)))
    return deg.value, rad.value, feat


def mlp_forward(params, X, out, stream=None) -> None:
    _check(lib().fd_mlp_forward(C.c_void_p(params.data_ptr()), X.shape[0], C.c_void_p(X.data_ptr()),
                                C.c_void_p(out.data_ptr()), _stream(stream)))


def mlp_grad(params, X, Y, w, G, loss, stream=None) -> None:
    _check(lib().fd_mlp_grad(C.c_void_p(params.data_ptr()), X.shape[0], C.c_void_p(X.data_ptr()),
                             C.c_void_p(Y.data_ptr()), C.c_void_p(w.data_ptr()), C.c_void_p(G.data_ptr()),
                             C.c_void_p(loss.data_ptr()), _stream(stream)))


def mlp_adam(params, G, M, V, step: int, lr: float, wd: float = 0.0, stream=None) -> None:
    _check(lib().fd_mlp_adam(C.c_void_p(params.data_ptr()), C.c_void_p(G.data_ptr()), C.c_void_p(M.data_ptr()),
                             C.c_void_p(V.data_ptr()), step, lr, wd, _stream(stream)))


def window_count(mu_kpm: np.ndarray, D: int, a: float, b: float, damped: bool = False) -> float:
    """fd_kpm_count: estimated number of eigenvalues in the scaled window
    [a, b] from KPM moments (damped: the moments carry the Jackson factors)."""
    mu = np.ascontiguousarray(mu_kpm, dtype=np.float64)
    out = _D()
    _check(lib().fd_kpm_count(mu.ctypes.data, mu.size, int(damped), D, a, b, C.byref(out)))
    return out.value


def autotune(m: "Matrix", dtype: str = "f64", nb: int = 64, stream=None) -> tuple:
    """Pick the fastest launch shape of the fused step for (m, dtype, nb)."""
    shape = (C.c_int32 * 10)()
    _check(lib().fd_autotune(m.handle, FD_F64 if dtype == "f64" else FD_F32, nb, shape, _stream(stream)))
    return tuple(shape)


def stream(op: int, a, c, b=None, scalar: float = 0.0, stream=None) -> None:
    """op 0: c = a; op 1: c = a + scalar b (1-D float64 GPU tensors)."""
    _check(lib().fd_stream(op, a.numel(), C.c_void_p(a.data_ptr()),
                           C.c_void_p(b.data_ptr()) if b is not None else None,
                           C.c_void_p(c.data_ptr()), scalar, _stream(stream)))


def lehmann(V, W, rho: float, stream=None):
    """Lehmann bounds (fd_lehmann) for the shift rho from V and W = A V (GPU
    float64 D x n blocks with one leading dimension): (lower, upper) numpy
    arrays; [lower[i], rho) and (rho, upper[i]] each hold at least i+1
    eigenvalues."""
    pv, ld, dt = _blk(V, "V")
    pw, ldw, dtw = _blk(W, "W")
    if dt != FD_F64 or dtw != FD_F64 or ld != ldw or V.shape != W.shape:
        raise ValueError("V and W must be float64 blocks of one shape and leading dimension")
    n = V.shape[1]
    lo = np.empty(n)
    up = np.empty(n)
    nl, nu = _I32(), _I32()
    _check(lib().fd_lehmann(V.shape[0], n, pv, pw, ld, rho, lo.ctypes.data, C.byref(nl), up.ctypes.data,
                            C.byref(nu), _stream(stream)))
    return lo[:nl.value].copy(), up[:nu.value].copy()


def lanczos(m: Matrix, k: int = 40, seed: int = 1, stream=None):
    """fd_lanczos: (theta ascending, residual bounds) of k Lanczos steps."""
    th = np.empty(k)
    rs = np.empty(k)
    n = _I32()
    _check(lib().fd_lanczos(m.handle, k, seed, th.ctypes.data, rs.ctypes.data, C.byref(n), _stream(stream)))
    return th[:n.value].copy(), rs[:n.value].copy()


def debug_alloc_limit(nbytes: int) -> None:
    """fd_debug_alloc_limit: make solver buffers above nbytes fail (0: off)."""
    _check(lib().fd_debug_alloc_limit(nbytes))


def syev_last_sweeps() -> int:
    return int(lib().fd_syev_last_sweeps())


def orthog(V, method: int = FD_ORTHO_SVQB2, seed: int = 0, stream=None) -> int:
    pv, ldv, _ = _blk(V, "V")
    r = _I32()
    _check(lib().fd_orthog(V.shape[0], V.shape[1], pv, ldv, method, seed, C.byref(r), _stream(stream)))
    return r.value


def rayleigh_ritz(m: Matrix, V, W, nb: int, stream=None):
    pv, ld, _ = _blk(V, "V")
    pw, ldw, _ = _blk(W, "W")
    if ld != ldw:
        raise ValueError("V and W must share a leading dimension")
    ns = V.shape[1]
    th = np.empty(ns)
    rho = np.empty(ns)
    _check(lib().fd_rayleigh_ritz(m.handle, ns, nb, pv, pw, ld, th.ctypes.data, rho.ctypes.data, _stream(stream)))
    return th, rho


@dataclass
class SolveResult:
    status: int
    evals: np.ndarray
    resid: np.ndarray
    evecs: object
    stats: dict


def solve(m: Matrix, tau_lo: float, tau_hi: float, n_target: int, n_search: int, nb: int, degree: int,
          max_iter: int = 50, tol: float = 1e-9, precision: int = 0, ortho: int = FD_ORTHO_SVQB2,
          seed: int = 0, V0: np.ndarray | None = None, want_vectors: bool = True,
          adapt: int = 0, picker=None, interval: int = 0) -> SolveResult:
    """fd_solve; V0 is a host D x n_search float64 array (or None).  degree 0
    picks the degree from KPM moments (picker: GPU float32 parameter tensor
    of the degree-picker network, or None for the plain rule)."""
    import torch
    p = SolveParams(tau_lo, tau_hi, n_target, n_search, nb, degree, max_iter, tol, precision, ortho, seed, adapt,
                    C.c_void_p(picker.data_ptr()) if picker is not None else None, interval)
    ev = np.full(n_target, np.nan)
    rs = np.full(n_target, np.nan)
    vecs = torch.empty((m.D, n_target), dtype=torch.float64, device="cuda") if want_vectors else None
    v0p = None
    if V0 is not None:
        V0 = np.ascontiguousarray(V0, dtype=np.float64)
        if V0.shape != (m.D, n_search):
            raise ValueError("V0 must be D x n_search")
        v0p = V0.ctypes.data
    st = SolveStats()
    torch.cuda.synchronize()
    status = _check(lib().fd_solve(m.handle, C.byref(p), v0p, ev.ctypes.data,
                                   vecs.data_ptr() if vecs is not None else None, rs.ctypes.data,
                                   C.byref(st)), allow=(FD_OK, FD_ERR_NOT_CONVERGED))
    return SolveResult(status, ev, rs, vecs, st.as_dict())


# ------------------------------------------------------------------- batched --
class Batch:
    """Owning wrapper of an fd_batch handle: the instance matrices stacked as
    one block-diagonal CSR on the GPU (instance i owns rows off[i]:off[i+1])."""

    def __init__(self, mats):
        arr = (C.c_void_p * len(mats))(*[m.handle for m in mats])
        h = C.c_void_p()
        _check(lib().fd_batch_create(len(mats), arr, C.byref(h)))
        self._h = h
        self.n = len(mats)
        D = _I64()
        off = np.empty(self.n + 1, np.int64)
        _check(lib().fd_batch_info(self._h, C.byref(D), off.ctypes.data))
        self.D, self.off = D.value, off
        self.lam = [(m.lam_lo, m.lam_hi) for m in mats]

    @property
    def handle(self):
        return self._h

    def __del__(self):
        try:
            if self._h:
                lib().fd_batch_free(self._h)
                self._h = None
        except Exception:
            pass


def batch_autotune(b: Batch, dtype: str = "f64", nb: int = 0, stream=None) -> tuple:
    """fd_batch_autotune: (nb, chunk rows, entry loop) chosen for the batch."""
    shape = (C.c_int32 * 3)()
    _check(lib().fd_batch_autotune(b.handle, FD_F64 if dtype == "f64" else FD_F32, nb, shape, _stream(stream)))
    return tuple(shape)


def batch_spmmv(b: Batch, X, Y, stream=None) -> None:
    """Y = A_i X on every instance's rows (fd_batch_spmmv)."""
    px, ldx, dt = _blk(X, "X")
    py, ldy, dty = _blk(Y, "Y")
    if dt != dty or X.shape != Y.shape or X.shape[0] != b.D:
        raise ValueError("X and Y must be D_total x nb blocks of one dtype")
    _check(lib().fd_batch_spmmv(b.handle, dt, X.shape[1], px, ldx, py, ldy, _stream(stream)))


def batch_filter(b: Batch, V, mu, degree, alpha, beta, W1, W2, nb: int, use_graph: bool = True,
                 stream=None) -> None:
    """fd_batch_filter: mu is a list of per-instance coefficient arrays (the
    length of mu[i] minus one is instance i's degree, 0 entries: idle)."""
    pv, ldv, dt = _blk(V, "V")
    p1, ldw, _ = _blk(W1, "W1")
    p2, ldw2, _ = _blk(W2, "W2")
    if ldw != ldw2 or V.shape[1] % nb:
        raise ValueError("W1 and W2 need one leading dimension; V's width a multiple of nb")
    dmax = max(int(d) for d in degree)
    M = np.zeros((b.n, dmax + 1))
    for i, m in enumerate(mu):
        m = np.asarray(m, dtype=np.float64)
        M[i, :m.size] = m
    deg = np.ascontiguousarray(degree, dtype=np.int32)
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    be = np.ascontiguousarray(beta, dtype=np.float64)
    _check(lib().fd_batch_filter(b.handle, dt, nb, V.shape[1] // nb, pv, ldv, M.ctypes.data, deg.ctypes.data,
                                 dmax, al.ctypes.data, be.ctypes.data, p1, p2, ldw, int(use_graph),
                                 _stream(stream)))


class BatchResult:
    def __init__(self, status, evals, resid, evecs, stats, bstats):
        self.status, self.evals, self.resid, self.evecs = status, evals, resid, evecs
        self.stats, self.bstats = stats, bstats


def solve_batch(b: Batch, params: list, V0: np.ndarray | None = None, want_vectors: bool = False) -> BatchResult:
    """fd_solve_batch.  params: one dict per instance with the keys of
    solve() (tau_lo, tau_hi, n_target, n_search, nb, degree, max_iter, tol,
    seed, adapt; precision 0)."""
    import torch
    P = (SolveParams * b.n)()
    for i, q in enumerate(params):
        P[i] = SolveParams(q["tau_lo"], q["tau_hi"], q["n_target"], q["n_search"], q["nb"], q["degree"],
                           q.get("max_iter", 50), q.get("tol", 1e-9), 0, q.get("ortho", FD_ORTHO_SVQB2),
                           q.get("seed", 0), q.get("adapt", 0), None)
    nt = params[0]["n_target"]
    ev = np.full((b.n, nt), np.nan)
    rs = np.full((b.n, nt), np.nan)
    vecs = torch.empty((b.D, nt), dtype=torch.float64, device="cuda") if want_vectors else None
    v0p = None
    if V0 is not None:
        V0 = np.ascontiguousarray(V0, dtype=np.float64)
        if V0.shape != (b.D, params[0]["n_search"]):
            raise ValueError("V0 must be D_total x n_search")
        v0p = V0.ctypes.data
    st = (SolveStats * b.n)()
    bs = BatchStats()
    torch.cuda.synchronize()
    status = _check(lib().fd_solve_batch(b.handle, P, v0p, ev.ctypes.data,
                                         vecs.data_ptr() if vecs is not None else None, rs.ctypes.data,
                                         st, C.byref(bs)), allow=(FD_OK, FD_ERR_NOT_CONVERGED))
    return BatchResult(status, ev, rs, vecs, [x.as_dict() for x in st], bs.as_dict())
